"""Plain FP64 CPU oracle (ctypes wrapper over ``liboracle.so``).

TEST INFRASTRUCTURE ONLY: the tests, ``__graft_entry__.smoke()`` and the CPU
baseline leg of ``bench.py`` use it; the product library never imports it.
It shares no code with the HIP path.  The C source follows the paper
(TARTARUS) section by section; see the header comment of tartarus_oracle.c.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tartarus_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# The same source built with FMA contraction: a second correct FP64 rounding of
# the same arithmetic, used to measure how far rounding alone moves a result.
_LIB_FMA = os.path.join(_HERE, "liboracle_fma.so")

ESCAPED, CAPTURED, FAILED, ON_DISK = 0, 1, 2, 3


def build(force: bool = True, fma: bool = False) -> str:
    """Compile the oracle with plain IEEE semantics (no fast-math, no FMA
    contraction); ``fma=True`` builds the rounding variant with a*b+c fused."""
    out = _LIB_FMA if fma else _LIB
    if force or not os.path.exists(out):
        contract = ["-ffp-contract=fast", "-mfma"] if fma else ["-ffp-contract=off"]
        cmd = ["gcc", "-O2", "-fno-fast-math", *contract, "-fopenmp", "-std=c11",
               "-D_DEFAULT_SOURCE", "-Wall", "-shared", "-fPIC", _SRC, "-o", out, "-lm"]
        subprocess.run(cmd, check=True)
    return out


class Metric(C.Structure):
    _fields_ = [("kind", C.c_int), ("a", C.c_double), ("table", C.POINTER(C.c_double)),
                ("nr", C.c_int), ("nth", C.c_int), ("r_min", C.c_double), ("r_max", C.c_double)]


class Camera(C.Structure):
    _fields_ = [("r_obs", C.c_double), ("theta_obs", C.c_double), ("nx", C.c_int), ("ny", C.c_int),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double),
                ("beta_min", C.c_double), ("beta_max", C.c_double)]


class Disk(C.Structure):
    _fields_ = [("r_in", C.c_double), ("r_out", C.c_double), ("max_hits", C.c_int), ("opaque", C.c_int),
                ("shading", C.c_int)]


class Solver(C.Structure):
    _fields_ = [("rtol", C.c_double), ("atol", C.c_double), ("h0_frac", C.c_double),
                ("horizon_factor", C.c_double), ("r_escape", C.c_double), ("event_tol", C.c_double),
                ("max_steps", C.c_int64), ("method", C.c_int32), ("pad", C.c_int32)]


class Outputs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in (
        "cls", "n_hits", "final_rtp", "h_drift", "h_gate", "hit_r", "hit_g", "hit_flux",
        "hit_lambda", "hit_order", "intensity", "n_accept", "n_reject", "n_cross")]


_lib = None
USER_RHS = C.CFUNCTYPE(None, C.POINTER(C.c_double), C.POINTER(C.c_double), C.c_int)


_lib_fma = None


def lib(fma: bool = False):
    global _lib, _lib_fma
    if fma:
        if _lib_fma is None:
            if not os.path.exists(_LIB_FMA):
                build(fma=True)
            _lib_fma = _declare(C.CDLL(_LIB_FMA))
        return _lib_fma
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = _declare(C.CDLL(_LIB))
    return _lib


def _declare(L):
    dp = C.POINTER(C.c_double)
    L.or_trace.argtypes = [C.POINTER(Metric), C.POINTER(Camera), C.c_int, C.POINTER(Disk),
                           C.POINTER(Solver), C.POINTER(C.c_int64), C.c_int64,
                           C.POINTER(Outputs), C.c_int]
    L.or_hamiltonian.argtypes = [C.POINTER(Metric), dp]
    L.or_hamiltonian.restype = C.c_double
    L.or_rhs.argtypes = [C.POINTER(Metric), dp, dp]
    L.or_metric_eval.argtypes = [C.POINTER(Metric), C.c_double, C.c_double, dp, dp, dp]
    L.or_kerr_smooth_components.argtypes = [C.c_double, C.c_double, C.c_double, dp]
    L.or_initial_state.argtypes = [C.POINTER(Metric), C.POINTER(Camera), C.c_int, C.c_int, dp]
    L.or_horizon.argtypes = [C.c_double]
    L.or_horizon.restype = C.c_double
    L.or_isco.argtypes = [C.c_double]
    L.or_isco.restype = C.c_double
    L.or_nt_flux.argtypes = [C.c_double] * 4
    L.or_nt_flux.restype = C.c_double
    L.or_redshift.argtypes = [C.c_double] * 4
    L.or_redshift.restype = C.c_double
    L.or_dp45_tableau.argtypes = [dp, dp, dp, dp]
    L.or_dp45_fixed.argtypes = [C.c_int, USER_RHS, dp, C.c_double, C.c_int, dp]
    L.or_rk_tableau.argtypes = [C.c_int, dp, dp, dp, dp]
    L.or_rk_fixed.argtypes = [C.c_int, C.c_int, USER_RHS, dp, C.c_double, C.c_int, dp]
    L.or_gbs_fixed.argtypes = [C.c_int, C.c_int, USER_RHS, dp, C.c_double, C.c_int, dp]
    L.or_gbs_columns.restype = C.c_int
    L.or_verlet_fixed.argtypes = [C.c_int, USER_RHS, dp, C.c_double, C.c_int]
    L.or_verlet_fixed.restype = C.c_int
    L.or_hermite.argtypes = [C.c_double] * 6
    L.or_hermite.restype = C.c_double
    L.or_bisect_count.argtypes = [C.c_double, C.c_double]
    L.or_bisect_count.restype = C.c_int
    L.or_build_kerr_table.argtypes = [C.c_double, C.c_int, C.c_int, C.c_double, C.c_double, dp]
    L.or_max_threads.restype = C.c_int
    L.or_trace_path.argtypes = [C.POINTER(Metric), dp, C.c_double, C.POINTER(Disk), C.POINTER(Solver),
                                dp, dp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), dp]
    L.or_rk4_step.argtypes = [C.POINTER(Metric), dp, C.c_double, dp]
    L.or_rk4_run.argtypes = [C.POINTER(Metric), dp, C.c_double, C.c_double, C.c_double, C.c_int, C.c_int]
    L.or_rk4_run.restype = C.c_int
    return L


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_metric(a: float, table: np.ndarray | None = None, nr=0, nth=0, r_min=0.0, r_max=0.0) -> Metric:
    m = Metric()
    m.kind = 0 if table is None else 1
    m.a = float(a)
    if table is not None:
        m.table = _dptr(table)
        m.nr, m.nth, m.r_min, m.r_max = int(nr), int(nth), float(r_min), float(r_max)
        m._keep = table  # keep the array alive with the struct
    return m


def make_camera(c: dict) -> Camera:
    return Camera(c["r_obs"], c["theta_obs"], c["nx"], c["ny"], c["alpha_min"], c["alpha_max"],
                  c["beta_min"], c["beta_max"])


def make_disk(d: dict | None) -> Disk:
    if d is None:
        return Disk(0.0, 0.0, 0, 0, 0)
    return Disk(d.get("r_in", 0.0), d["r_out"], d.get("max_hits", 3), d.get("opaque", 0), d.get("shading", 0))


def make_solver(s: dict) -> Solver:
    return Solver(s["rtol"], s["atol"], s.get("h0_frac", 0.01), s.get("horizon_factor", 1.01),
                  s["r_escape"], s.get("event_tol", 1e-12), s.get("max_steps", 1_000_000), s.get("method", 0), 0)


def alloc_outputs(n: int) -> dict:
    o = {
        "cls": np.zeros(n, np.int32), "n_hits": np.zeros(n, np.int32),
        "final_rtp": np.zeros((n, 3)), "h_drift": np.zeros(n), "h_gate": np.zeros(n),
        "hit_r": np.zeros((n, 3)), "hit_g": np.zeros((n, 3)), "hit_flux": np.zeros((n, 3)),
        "hit_lambda": np.zeros((n, 3)), "hit_order": np.zeros((n, 3), np.int32),
        "intensity": np.zeros(n), "n_accept": np.zeros(n, np.int32),
        "n_reject": np.zeros(n, np.int32), "n_cross": np.zeros(n, np.int32),
    }
    return o


def trace(metric: Metric, cameras, disk: Disk, solver: Solver, ray_ids=None, threads: int = 0,
          fma: bool = False) -> dict:
    """Trace rays; ``cameras`` is one Camera or a list (all with the same nx, ny).
    ``fma=True`` runs the FMA-contracted build of the same source."""
    L = lib(fma)
    if isinstance(cameras, Camera):
        cameras = [cameras]
    cams = (Camera * len(cameras))(*cameras)
    per = cameras[0].nx * cameras[0].ny
    if ray_ids is None:
        n = per * len(cameras)
        ids_p = None
    else:
        ray_ids = np.ascontiguousarray(ray_ids, dtype=np.int64)
        n = len(ray_ids)
        ids_p = ray_ids.ctypes.data_as(C.POINTER(C.c_int64))
    o = alloc_outputs(n)
    so = Outputs(*[o[f].ctypes.data for f, _ in Outputs._fields_])
    L.or_trace(C.byref(metric), cams, len(cameras), C.byref(disk), C.byref(solver), ids_p, n,
               C.byref(so), int(threads))
    return o


def initial_state(metric: Metric, camera: Camera, i: int, j: int) -> np.ndarray:
    q = np.zeros(8)
    lib().or_initial_state(C.byref(metric), C.byref(camera), i, j, _dptr(q))
    return q


def hamiltonian(metric: Metric, q) -> float:
    q = np.ascontiguousarray(q, dtype=np.float64)
    return lib().or_hamiltonian(C.byref(metric), _dptr(q))


def rhs(metric: Metric, q) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    d = np.zeros(8)
    lib().or_rhs(C.byref(metric), _dptr(q), _dptr(d))
    return d


def metric_eval(metric: Metric, r: float, th: float):
    g, gr, gt = np.zeros(5), np.zeros(5), np.zeros(5)
    lib().or_metric_eval(C.byref(metric), r, th, _dptr(g), _dptr(gr), _dptr(gt))
    return g, gr, gt


def kerr_smooth_components(a: float, r: float, th: float) -> np.ndarray:
    out = np.zeros((5, 4))
    lib().or_kerr_smooth_components(a, r, th, _dptr(out))
    return out


def build_kerr_table(a: float, nr: int, nth: int, r_min: float, r_max: float) -> np.ndarray:
    t = np.zeros((5, nr, nth, 4))
    lib().or_build_kerr_table(a, nr, nth, r_min, r_max, _dptr(t))
    return t


def horizon(a): return lib().or_horizon(a)
def isco(a): return lib().or_isco(a)
def nt_flux(a, r_in, r_out, r): return lib().or_nt_flux(a, r_in, r_out, r)
def redshift(a, r, p_t, p_phi): return lib().or_redshift(a, r, p_t, p_phi)
def hermite(s, y0, d0, y1, d1, h): return lib().or_hermite(s, y0, d0, y1, d1, h)
def bisect_count(h, tol): return lib().or_bisect_count(h, tol)
def max_threads(): return lib().or_max_threads()


METHODS = {"dp45": 0, "ck45": 1, "rkf45": 2, "gbs": 3, "verlet": 4}
RK_METHODS = {"dp45": 0, "ck45": 1, "rkf45": 2}


def dp45_tableau():
    return rk_tableau(0)


def rk_tableau(method: int):
    """(c, a[7][6], b, b*) of a 5(4) pair: 0 Dormand-Prince, 1 Cash-Karp, 2 Fehlberg."""
    c, a, b, bs = np.zeros(7), np.zeros(42), np.zeros(7), np.zeros(7)
    lib().or_rk_tableau(method, _dptr(c), _dptr(a), _dptr(b), _dptr(bs))
    return c, a.reshape(7, 6), b, bs


def dp45_fixed(f, y0, h: float, nsteps: int):
    return rk_fixed(0, f, y0, h, nsteps)


def _user_rhs(f):
    def cb(yp, dyp, nn):
        y = np.ctypeslib.as_array(yp, shape=(nn,)).copy()
        d = f(y)
        for k in range(nn):
            dyp[k] = float(d[k])
    return USER_RHS(cb)


def rk_fixed(method: int, f, y0, h: float, nsteps: int):
    """Fixed-step steps of a 5(4) pair on y' = f(y) (f: numpy array -> numpy array); returns
    (y, last error vector)."""
    n = len(y0)
    cfun = _user_rhs(f)
    y = np.ascontiguousarray(y0, dtype=np.float64).copy()
    e = np.zeros(n)
    lib().or_rk_fixed(method, n, cfun, _dptr(y), h, nsteps, _dptr(e))
    return y, e


def verlet_fixed(f, y0, h: float, nsteps: int):
    """nsteps fixed Verlet steps on a Hamiltonian system y = [x, p] with
    f(y) = [dH/dp, -dH/dx]; returns (y, steps completed)."""
    n = len(y0)
    assert n % 2 == 0 and n <= 16
    cfun = _user_rhs(f)
    y = np.ascontiguousarray(y0, dtype=np.float64).copy()
    done = lib().or_verlet_fixed(n, cfun, _dptr(y), h, nsteps)
    return y, done


def gbs_columns() -> int:
    """Extrapolation columns K the ray tracer uses with method 3."""
    return lib().or_gbs_columns()


def gbs_fixed(K: int, f, y0, h: float, nsteps: int):
    """Fixed macro-steps of Gragg-Bulirsch-Stoer extrapolation with K columns
    (2 <= K <= 8) on y' = f(y); returns (y, last error vector)."""
    assert 2 <= K <= 8
    n = len(y0)
    cfun = _user_rhs(f)
    y = np.ascontiguousarray(y0, dtype=np.float64).copy()
    e = np.zeros(n)
    lib().or_gbs_fixed(K, n, cfun, _dptr(y), h, nsteps, _dptr(e))
    return y, e


def trace_path(metric: Metric, q0, h0: float, disk: Disk, solver: Solver, cap: int = 200000) -> dict:
    """One ray from state q0 with its accepted states recorded (initial state first)."""
    q0 = np.ascontiguousarray(q0, dtype=np.float64)
    states = np.zeros((cap, 8))
    lam = np.zeros(cap)
    n = C.c_int(0)
    res = (C.c_int * 5)()
    resd = np.zeros(18)
    lib().or_trace_path(C.byref(metric), _dptr(q0), h0, C.byref(disk), C.byref(solver), _dptr(states),
                        _dptr(lam), cap, C.byref(n), res, _dptr(resd))
    k = n.value
    return dict(states=states[:k], lam=lam[:k], cls=res[0], n_hits=res[1], n_accept=res[2],
                n_reject=res[3], n_cross=res[4], final_rtp=resd[0:3].copy(), h_drift=resd[3],
                h_gate=resd[4], intensity=resd[5], hit_r=resd[6:9].copy(), hit_g=resd[9:12].copy(),
                hit_flux=resd[12:15].copy(), hit_lambda=resd[15:18].copy())


def rk4_step(metric: Metric, q, h: float) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros(8)
    lib().or_rk4_step(C.byref(metric), _dptr(q), h, _dptr(out))
    return out


def rk4_run(metric: Metric, q, h_frac: float, r_lo: float, r_hi: float, max_steps: int, stop_on_equator: bool):
    """Advance q in place with RK4 steps of h_frac * r; returns (q, steps taken)."""
    q = np.ascontiguousarray(q, dtype=np.float64).copy()
    n = lib().or_rk4_run(C.byref(metric), _dptr(q), h_frac, r_lo, r_hi, max_steps, int(stop_on_equator))
    return q, n
