#!/usr/bin/env python3
"""Benchmark of the Kerr null-geodesic tracer on one MI355X.

Workload: Kerr a = 0.9, observer at r = 1000 M and 60 deg inclination, a
512 x 512 camera over alpha, beta in [-25, 25] M, a Novikov-Thorne disk from
r_ISCO to 20 M with up to 3 recorded crossings (synthetic camera grid, no
data).  One "step" is one full trace of the image (camera initial conditions,
Dormand-Prince 5(4) integration, events, shading) through the C ABI; inputs
are generated on the device, so the timed region reads nothing from the host.

The headline value is FP64 rays/s at the tolerance where the constraint gate
|H| <= 1e-8 holds for every ray (rtol = 3e-10, atol = 3e-12; checked on the
run's own outputs).  Extra legs report FP64 and mixed precision at rtol = 1e-8.
The roofline entry prices the integrator kernel's algorithmic FP64 work
(per-ray attempt counts x FLOPs per attempt) against the FP64 vector peak.
The CPU baseline is the plain FP64 oracle on a seeded sample of the same
image's pixels, on all host cores.

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
GATE_RTOL, GATE_ATOL = 3e-10, 3e-12
PEAK_FP64_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP32_TFLOPS = 78.6     # non-packed FP32 (packed FP32 is disabled in this build)

# Algorithmic FLOPs (FMA = 2, division / sqrt / transcendental = 1) of the
# analytic-Kerr FP64 path, counted from the formulas the kernel evaluates:
FLOP_RHS = 72               # one right-hand side incl. H
FLOP_ATTEMPT = 6 * FLOP_RHS + 140 + 66 + 72 + 38 + 5 + 6   # stages, y5, error, norm, controller, events = 759
FLOP_RAY_INIT = 130         # observer metric, tetrad, first right-hand side
FLOP_EVENT = 300            # Hermite set-up + ~40 bisection iterations
FLOP_HIT = 120              # Omega, u^t, g, Page-Thorne flux


def algorithmic_flops(out: dict) -> float:
    att = out["n_accept"].astype(np.float64) + out["n_reject"]
    return float(att.sum() * FLOP_ATTEMPT + len(att) * (FLOP_RAY_INIT + FLOP_EVENT)
                 + out["n_cross"].sum() * FLOP_EVENT + out["n_hits"].sum() * FLOP_HIT)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


SHAPE_KEYS = ("block_threads", "blocks_per_cu", "chunk", "refill_min", "order")
HERE = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_FILE = os.path.join(HERE, "profiles", "trace_persistent_fp64_kerr09_512.traffic.json")


_COMMENT = re.compile(r"//[^\n]*|/\*.*?\*/", re.S)


def kernel_source_hash() -> str:
    """sha256 over the device sources with comments and blank lines removed;
    HBM traffic measured for other code is stale."""
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(HERE, "paper_2609_08989_amd", "csrc", "*.h*"))):
        h.update(os.path.basename(f).encode())
        with open(f, encoding="utf-8") as fh:
            code = _COMMENT.sub("", fh.read())
        h.update("\n".join(ln.rstrip() for ln in code.splitlines() if ln.strip()).encode())
    return h.hexdigest()


def _committed_counters():
    """The headline kernel's committed rocprofv3 figures, if they were taken on
    these kernel sources; else None."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except OSError:
        return None
    return t if t.get("source_sha256") == kernel_source_hash() else None


def measured_traffic():
    """HBM bytes per launch of the headline kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE runs (copy-calibrated), if they were taken on these
    kernel sources; else None.  The bytes are the per-ray records, outputs and
    job tables of the image, which do not depend on the launch shape; the
    shape they were measured at is returned with them."""
    t = _committed_counters()
    if t is None:
        return None, None
    return float(t["fetch_bytes"] + t["write_bytes"]), t.get("launch")


def attempts_histogram(att) -> dict:
    """Attempted steps per ray: quantiles and counts per power-of-two bin
    (key k counts rays with 2^k <= attempts < 2^(k+1))."""
    import numpy as np
    att = np.asarray(att, dtype=np.int64)
    q = {f"p{p}": float(np.percentile(att, p)) for p in (0, 10, 50, 90, 99, 100)}
    k = np.floor(np.log2(np.maximum(att, 1))).astype(int)
    q["log2_bins"] = {str(int(b)): int(c) for b, c in zip(*np.unique(k, return_counts=True))}
    return q


def shape(L):
    return [L.block_threads, L.blocks_per_cu, L.chunk, L.refill_min, L.order]


def time_leg(T, torch, args_tuple, out, steps, warmup, launch=None):
    """Wall time of `steps` traces (bracketed by device synchronizations), and
    the mean duration of their integrator launches, from the HIP event pair the
    library records around each one on the trace's stream."""
    for _ in range(warmup):
        T.tartarus_trace(*args_tuple, out, launch=launch)
    torch.cuda.synchronize()
    T.tartarus_kernel_time()                 # drop anything recorded before
    T.tartarus_kernel_timing(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        T.tartarus_trace(*args_tuple, out, launch=launch)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T.tartarus_kernel_timing(False)
    kernel_total_ms, launches = T.tartarus_kernel_time()
    assert launches == steps, (launches, steps)
    return wall, kernel_total_ms / launches


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


def cpu_baseline(w, solver, seconds: float) -> dict:
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
            "sample": f"{n} seeded-random pixels of the same 512x512 image (rtol={solver['rtol']:g}), "
                      f"plain FP64 C oracle, OpenMP over pixels, {dt:.1f} s"}


def workload_legs(T, torch, W, out_cache, steps: int = 2, autotune: bool = True) -> dict:
    """rays/s of the other image workloads (rtol 1e-8): the Schwarzschild
    shadow, the a = 0.998 2048^2 scene in FP64 and mixed, the paper's OSIRIS
    calibration scene, and the 64-camera tabulated-metric batch.  Each image
    scene is autotuned first (untimed); the tabulated batch (0.7 s a launch)
    uses the shape measured best for it (256 threads, 2 blocks per CU, pixel
    order)."""
    legs = {}
    for name, prec in (("schwarzschild_64", T.PREC_FP64), ("kerr0998_2048", T.PREC_FP64),
                       ("kerr0998_2048", T.PREC_MIXED), ("osiris_1024", T.PREC_FP64),
                       ("tabulated07_64cams", T.PREC_FP64)):
        w = W.WORKLOADS[name]
        cams = [T.make_camera(c) for c in w["cameras"]]
        n = sum(c["nx"] * c["ny"] for c in w["cameras"])
        if "table" in w:
            t = w["table"]
            r_min = t["r_min_over_rplus"] * (1.0 + np.sqrt(1.0 - w["a"] ** 2))
            tab = torch.zeros(5 * t["nr"] * t["nth"] * 4, dtype=torch.float64, device="cuda")
            T.tartarus_build_kerr_table(w["a"], t["nr"], t["nth"], r_min, t["r_max"], tab)
            metric = T.make_metric(w["a"], tab, t["nr"], t["nth"], r_min, t["r_max"])
        else:
            metric = T.make_metric(w["a"])
        if n not in out_cache:
            out_cache.clear()
            out_cache[n] = T.alloc_outputs(n)
        out = out_cache[n]
        la = (metric, cams, T.make_disk(w["disk"]), T.make_solver(w["solver"], prec))
        log("bench: workload", name, "mixed" if prec else "fp64")
        if "table" in w:
            launch = T.make_launch(256, 2, 1, 4, T.ORDER_PIXEL)
        elif autotune:
            launch = T.tartarus_autotune(*la, out)
        else:
            launch = None
        wl, km = time_leg(T, torch, la, out, steps, 1, launch)
        o = T.to_numpy(out)
        att = o["n_accept"] + o["n_reject"]
        legs[f"{name}_{'mixed' if prec else 'fp64'}"] = {
            "rays": n, "rays_per_s": n * steps / wl, "kernel_ms": km, "attempts_per_ray": float(att.mean()),
            "failed_rays": int((o["cls"] == 2).sum()),
            "launch": dict(zip(SHAPE_KEYS, shape(launch))) if launch is not None else "default"}
    return legs


def serving_leg(T, torch, W, n_requests: int, loads=(0.5, 0.8, 0.95), budget_gib: int = 8,
                arrival_order_load: float = 0.8) -> dict:
    """Poisson streams of image requests (resolution uniform over 64^2..1024^2,
    spin, inclination, disk size drawn per request) submitted at their arrival
    times through tartarus_submit under an HBM budget that makes admission
    bind; latency = done - submit per request.  The offered load is a fraction
    of the server's own throughput, measured first on a burst of requests from
    the same distribution (another seed); stream k uses seed k.  The queue
    hands out the smallest admitted request's rays first; one more stream, at
    arrival_order_load with the seed of that load, runs with arrival order for
    comparison."""
    mk = lambda r: (T.make_metric(r["a"]), T.make_camera(r["camera"]), T.make_disk(r["disk"]),
                    T.make_solver(r["solver"]))
    T.tartarus_shutdown()
    T.tartarus_init(0, budget_gib << 30)
    # capacity: a burst submitted at once
    burst = W.request_stream(1000, 48, 1e9)
    bouts = [T.alloc_outputs(r["camera"]["nx"] * r["camera"]["ny"]) for r in burst]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in [T.tartarus_submit(*mk(r), o) for r, o in zip(burst, bouts)]:
        T.tartarus_wait(t, 120000)
    capacity = sum(r["camera"]["nx"] * r["camera"]["ny"] for r in burst) / (time.perf_counter() - t0)
    del bouts
    mean_rays = float(np.mean([r * r for r in W.RESOLUTIONS]))
    runs = []
    plan = [(seed, load, T.SERVE_SMALLEST_FIRST) for seed, load in enumerate(loads)]
    if arrival_order_load in loads:
        plan.append((loads.index(arrival_order_load), arrival_order_load, T.SERVE_ARRIVAL))
    for seed, load, policy in plan:
        T.tartarus_serving_order(policy)
        rate = load * capacity / mean_rays
        reqs = W.request_stream(seed, n_requests, rate)
        outs = [T.alloc_outputs(r["camera"]["nx"] * r["camera"]["ny"]) for r in reqs]
        torch.cuda.synchronize()
        log("bench: serving load", load, "requests", n_requests, "order", policy)
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
        failed = int(sum(int((T.to_numpy({"cls": o["cls"]})["cls"] == 2).sum()) for o in outs))
        runs.append({"load": load, "seed": seed, "requests": len(reqs), "arrival_rate_per_s": rate,
                     "order": "smallest_first" if policy == T.SERVE_SMALLEST_FIRST else "arrival",
                     "p50_latency_ms": float(np.percentile(lat_ms[warm:], 50)),
                     "p99_latency_ms": float(np.percentile(lat_ms[warm:], 99)),
                     "max_latency_ms": float(lat_ms[warm:].max()), "rays_per_s": rays / span,
                     "failed_rays": failed})
        del outs
    T.tartarus_shutdown()
    T.tartarus_init(0, 0)
    T.tartarus_serving_order(T.SERVE_SMALLEST_FIRST)
    ref = min((x for x in runs if x["order"] == "smallest_first"), key=lambda x: abs(x["load"] - 0.8))
    return {"requests_per_load": n_requests, "capacity_rays_per_s": capacity, "precision": "fp64",
            "rtol": W.solver()["rtol"], "hbm_budget_gib": budget_gib,
            "p50_latency_ms": ref["p50_latency_ms"], "p99_latency_ms": ref["p99_latency_ms"], "load": ref["load"],
            "by_load": runs,
            "note": "latency = completion - submission; first 10 requests of each stream are warm-up; "
                    "load = fraction of the burst capacity; headline p50/p99 at load 0.8, smallest request first"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true", help="time only the headline leg")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-autotune", action="store_true", help="use the default launch shape")
    ap.add_argument("--launch", default="", help="force the launch shape block,blocks_per_cu,chunk,refill_min[,order]")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving-latency leg")
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
    w = W.WORKLOADS["kerr09_512"]
    cam = w["cameras"][0]
    n = cam["nx"] * cam["ny"]
    metric, cams, disk = T.make_metric(w["a"]), [T.make_camera(cam)], T.make_disk(w["disk"])
    gate_solver = dict(w["solver"], rtol=GATE_RTOL, atol=GATE_ATOL)
    out = T.alloc_outputs(n)

    # ---- headline: FP64 at the gate tolerance
    leg_args = (metric, cams, disk, T.make_solver(gate_solver, T.PREC_FP64))
    tuned = {}
    launch = None
    if args.launch:
        launch = T.make_launch(*[int(v) for v in args.launch.split(",")])
        tuned["fp64"] = shape(launch)
    elif not args.no_autotune:
        log("bench: autotune")
        # untimed: pick the launch shape for this workload (part of the warm-up)
        L = T.tartarus_autotune(*leg_args, out)
        tuned["fp64"] = shape(L)
    log("bench: headline leg (fp64, gate tolerance)", tuned)
    wall, kern_ms = time_leg(T, torch, leg_args, out, args.steps, args.warmup, launch)
    o = T.to_numpy(out)
    ms_per_step = wall * 1e3 / args.steps
    value = n * args.steps / wall
    h_gate_max = float(o["h_gate"][o["cls"] != 2].max())
    flops = algorithmic_flops(o)
    achieved = flops / (kern_ms * 1e-3) / 1e12
    att = o["n_accept"] + o["n_reject"]
    traffic_bytes, traffic_shape = measured_traffic()
    cnt = _committed_counters()
    executed = None
    if cnt is not None and cnt.get("executed_fp64_flop"):
        ex = float(cnt["executed_fp64_flop"])
        executed = {"flop_per_launch": ex, "achieved": ex / (kern_ms * 1e-3) / 1e12,
                    "frac": ex / (kern_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS,
                    "note": "FP64 VALU instructions x lanes x lane efficiency from the committed counters "
                            "(FMA = 2), over this run's kernel time"}
    sh0 = dict(zip(SHAPE_KEYS, tuned.get("fp64", [0, 0, 0, 0, 0])))
    launched = (sh0["block_threads"] // 64 * sh0["blocks_per_cu"] / 4.0
                if sh0["block_threads"] > 0 and sh0["blocks_per_cu"] > 0 else None)
    occupancy = {"launched_waves_per_simd": launched, "max_waves_per_simd": 2,
                 "mean_resident_waves_per_simd": (cnt or {}).get("mean_resident_waves_per_simd"),
                 "counter_launch_shape": (cnt or {}).get("launch")}
    result = {
        "metric": METRIC, "value": value, "unit": "rays/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "kerr_a0.9_i60deg_r1000_512x512_disk_isco_to_20M", "rays": n,
                   "rtol": GATE_RTOL, "atol": GATE_ATOL, "precision": "fp64",
                   "gate_h_max": h_gate_max, "gate_holds": bool(h_gate_max <= 1e-8),
                   "failed_rays": int((o["cls"] == 2).sum()), "attempts_per_ray": float(att.mean()),
                   "attempts_histogram": attempts_histogram(att)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": traffic_bytes, "traffic_launch_shape": traffic_shape,
                     "kernel": "trace_persistent<0,0> (analytic Kerr, FP64)",
                     "kernel_ms": kern_ms, "flop_per_launch": flops,
                     "flop_per_attempt": FLOP_ATTEMPT, "executed": executed, "occupancy": occupancy},
    }

    # ---- extra legs at the config tolerance rtol = 1e-8
    if not args.no_extra:
        legs = {}
        # the headline trace with the work queue in pixel order instead of cost order
        sh = dict(zip(SHAPE_KEYS, tuned.get("fp64", [0, 0, 0, 0, 0])))
        lp = T.make_launch(sh["block_threads"], sh["blocks_per_cu"], sh["chunk"], sh["refill_min"], T.ORDER_PIXEL)
        log("bench: leg gate_pixel_order")
        wl, km = time_leg(T, torch, leg_args, out, args.steps, args.warmup, lp)
        legs["gate_pixel_order"] = {"rays_per_s": n * args.steps / wl, "kernel_ms": km}
        for name, prec in (("fp64_rtol1e-8", T.PREC_FP64), ("mixed_rtol1e-8", T.PREC_MIXED)):
            la = (metric, cams, disk, T.make_solver(w["solver"], prec))
            log("bench: leg", name)
            if prec == T.PREC_MIXED and not args.no_autotune:
                L = T.tartarus_autotune(*la, out)
                tuned["mixed"] = shape(L)
            wl, km = time_leg(T, torch, la, out, args.steps, args.warmup)
            ol = T.to_numpy(out)
            attl = ol["n_accept"] + ol["n_reject"]
            legs[name] = {"rays_per_s": n * args.steps / wl, "kernel_ms": km,
                          "attempts_per_ray": float(attl.mean()),
                          "fp32_attempt_frac": float(ol["n_fp32"].sum() / attl.sum()),
                          "gate_frac_le_1e-8": float(np.mean(ol["h_gate"] <= 1e-8)),
                          "failed_rays": int((ol["cls"] == 2).sum())}
        # the other two 5(4) pairs of Sec. 3.2 on the same image, rtol 1e-8
        for mname, mcode in (("ck45", T.METHOD_CK45), ("rkf45", T.METHOD_RKF45)):
            la = (metric, cams, disk, T.make_solver(dict(w["solver"], method=mcode), T.PREC_FP64))
            log("bench: leg", mname)
            wl, km = time_leg(T, torch, la, out, args.steps, args.warmup)
            ol = T.to_numpy(out)
            attl = ol["n_accept"] + ol["n_reject"]
            legs[f"{mname}_rtol1e-8"] = {"rays_per_s": n * args.steps / wl, "kernel_ms": km,
                                         "attempts_per_ray": float(attl.mean()),
                                         "failed_rays": int((ol["cls"] == 2).sum())}
        # Gragg-Bulirsch-Stoer (Sec. 3.2) beside Dormand-Prince: at the config and
        # gate tolerances, and at rtol 1e-12 where its order-12 macro-steps pay
        for mname, sv in (("gbs_rtol1e-8", dict(w["solver"], method=T.METHOD_GBS)),
                          ("gbs_gate", dict(gate_solver, method=T.METHOD_GBS)),
                          ("gbs_rtol1e-12", dict(w["solver"], rtol=1e-12, atol=1e-14, method=T.METHOD_GBS)),
                          ("fp64_rtol1e-12", dict(w["solver"], rtol=1e-12, atol=1e-14))):
            la = (metric, cams, disk, T.make_solver(sv, T.PREC_FP64))
            log("bench: leg", mname)
            wl, km = time_leg(T, torch, la, out, args.steps, args.warmup)
            ol = T.to_numpy(out)
            attl = ol["n_accept"] + ol["n_reject"]
            legs[mname] = {"rays_per_s": n * args.steps / wl, "kernel_ms": km,
                           "attempts_per_ray": float(attl.mean()),
                           "h_gate_max": float(ol["h_gate"][ol["cls"] != 2].max()),
                           "failed_rays": int((ol["cls"] == 2).sum())}
        # fixed-step Verlet (Sec. 3.2): h = 0.01 on a 256^2 image of the same scene,
        # stop at 1.05 r_+ (where its implicit stages still converge), two launches
        wv = dict(cam, nx=256, ny=256)
        nv = wv["nx"] * wv["ny"]
        sv = dict(w["solver"], method=T.METHOD_VERLET, h0_frac=0.01 / wv["r_obs"], horizon_factor=1.05)
        la = (metric, [T.make_camera(wv)], disk, T.make_solver(sv, T.PREC_FP64))
        outv = T.alloc_outputs(nv)
        log("bench: leg verlet_h0.01_256")
        wl, km = time_leg(T, torch, la, outv, 2, 1)
        ol = T.to_numpy(outv)
        legs["verlet_h0.01_256"] = {"rays": nv, "rays_per_s": nv * 2 / wl, "kernel_ms": km,
                                    "steps_per_ray": float(ol["n_accept"].mean()),
                                    "steps_per_s": float(ol["n_accept"].sum()) * 2 / wl,
                                    "h_gate_max": float(ol["h_gate"][ol["cls"] != 2].max()),
                                    "failed_rays": int((ol["cls"] == 2).sum())}
        legs.update(workload_legs(T, torch, W, {}, autotune=not args.no_autotune))
        legs["mixed_over_fp64_same_rtol"] = legs["mixed_rtol1e-8"]["rays_per_s"] / legs["fp64_rtol1e-8"]["rays_per_s"]
        legs["mixed_rtol1e-8_over_fp64_gate"] = legs["mixed_rtol1e-8"]["rays_per_s"] / value
        result["legs"] = legs

    if not args.no_serving:
        log("bench: serving leg")
        result["serving"] = serving_leg(T, torch, W, n_requests=args.serving_requests)
    if tuned:
        result["launch_shape"] = {k: dict(zip(SHAPE_KEYS, v)) for k, v in tuned.items()}
    if not args.no_cpu:
        log("bench: cpu baseline")
        result["cpu_baseline"] = cpu_baseline(w, gate_solver, args.cpu_seconds)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
