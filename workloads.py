"""Synthetic workload definitions shared by the tests, the benchmark and the smoke check.

This module holds input parameters and the seeded request-stream generator
only: no part of the ray-tracing arithmetic.  Every image workload is a
deterministic camera grid (no random numbers); only the serving stream draws
random numbers, from ``numpy.random.Generator(PCG64(seed))``.

Image workloads (observer distance D = r_obs in units of M, angles in radians):

* ``schwarzschild_64``   a = 0, theta_obs = 90 deg, r_obs = 1000, 64 x 64 over
  [-10, 10]^2, stop at 1.01 r_+ or r = 1100, no disk.
* ``kerr09_512``         a = 0.9, theta_obs = 60 deg, r_obs = 1000, 512 x 512 over
  [-25, 25]^2, thin disk from r_ISCO to 20, up to 3 recorded crossings.
* ``kerr0998_2048``      a = 0.998, theta_obs = 17 deg, 2048 x 2048 over [-20, 20]^2,
  disk r_ISCO .. 30.
* ``tabulated07_64cams`` tabulated Kerr a = 0.7 on a 512 (log r, 1.1 r_+ .. 2000)
  x 256 (theta) grid; 64 cameras theta_obs = 10 + 70 c / 63 deg, 512 x 512 each
  over [-25, 25]^2; disk r_ISCO .. 20.
* ``osiris_1024``        a = 0.98, theta_obs = 90 deg, 1024 x 1024 over [-8, 8]^2
  (the paper's calibration scene, Sec. 4.3), no disk.
* ``schwarzschild_disk_100`` the scene of the paper's Table 1 (Sec. 4.3):
  Schwarzschild (a = 0) with a Novikov-Thorne disk seen from D = r_obs = 100;
  the paper leaves the inclination, window, disk size and tolerance unstated:
  theta_obs = 80 deg, 512 x 512 over [-22, 22]^2, disk r_ISCO (6 M) .. 20 M,
  escape at 1.1 r_obs = 110 M, rtol = 1e-8.

The solver defaults: rtol = 1e-8, atol = 1e-10, first step 0.01 r_obs, escape at
1.1 r_obs (1100 M), horizon stop at 1.01 r_+, event tolerance 1e-12 in lambda.
"""
from __future__ import annotations

import math

import numpy as np

DEG = math.pi / 180.0


def camera(r_obs, theta_deg, nx, ny, half_width, half_height=None):
    hh = half_width if half_height is None else half_height
    return dict(r_obs=float(r_obs), theta_obs=float(theta_deg) * DEG, nx=int(nx), ny=int(ny),
                alpha_min=-float(half_width), alpha_max=float(half_width),
                beta_min=-float(hh), beta_max=float(hh))


def solver(rtol=1e-8, atol=1e-10, r_escape=1100.0, max_steps=1_000_000, **kw):
    s = dict(rtol=rtol, atol=atol, h0_frac=0.01, horizon_factor=1.01, r_escape=r_escape,
             event_tol=1e-12, max_steps=max_steps)
    s.update(kw)
    return s


WORKLOADS = {
    "schwarzschild_64": dict(
        a=0.0, cameras=[camera(1000.0, 90.0, 64, 64, 10.0)], disk=None, solver=solver()),
    "kerr09_512": dict(
        a=0.9, cameras=[camera(1000.0, 60.0, 512, 512, 25.0)],
        disk=dict(r_in=0.0, r_out=20.0, max_hits=3), solver=solver()),
    "kerr0998_2048": dict(
        a=0.998, cameras=[camera(1000.0, 17.0, 2048, 2048, 20.0)],
        disk=dict(r_in=0.0, r_out=30.0, max_hits=3), solver=solver()),
    "tabulated07_64cams": dict(
        a=0.7, cameras=[camera(1000.0, 10.0 + 70.0 * c / 63.0, 512, 512, 25.0) for c in range(64)],
        disk=dict(r_in=0.0, r_out=20.0, max_hits=3), solver=solver(),
        table=dict(nr=512, nth=256, r_min_over_rplus=1.1, r_max=2000.0)),
    "osiris_1024": dict(
        a=0.98, cameras=[camera(1000.0, 90.0, 1024, 1024, 8.0)], disk=None, solver=solver()),
    "schwarzschild_disk_100": dict(
        a=0.0, cameras=[camera(100.0, 80.0, 512, 512, 22.0)],
        disk=dict(r_in=0.0, r_out=20.0, max_hits=3), solver=solver(r_escape=110.0)),
}


def scaled(name: str, nx: int, ny: int | None = None, ncams: int | None = None) -> dict:
    """The named workload with its camera grid resampled to nx x ny (same window)."""
    w = dict(WORKLOADS[name])
    ny = nx if ny is None else ny
    cams = w["cameras"] if ncams is None else w["cameras"][:: max(1, len(w["cameras"]) // ncams)][:ncams]
    w["cameras"] = [dict(c, nx=nx, ny=ny) for c in cams]
    return w


# ---------------------------------------------------------------------------
# Serving stream: Poisson arrivals of mixed image requests (seeded).
# Draw order per request: inter-arrival, resolution, spin, inclination, outer radius.
# ---------------------------------------------------------------------------
RESOLUTIONS = (64, 128, 256, 512, 1024)


def request_stream(seed: int, n_requests: int, rate_per_s: float, resolutions=RESOLUTIONS):
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        res = int(resolutions[rng.integers(0, len(resolutions))])
        a = float(rng.uniform(0.0, 0.998))
        inc = float(rng.uniform(5.0, 85.0))
        r_out = float(rng.uniform(15.0, 50.0))
        out.append(dict(
            id=k, arrival_s=t, a=a,
            camera=camera(1000.0, inc, res, res, r_out),
            disk=dict(r_in=0.0, r_out=r_out, max_hits=3),
            solver=solver()))
    return out
