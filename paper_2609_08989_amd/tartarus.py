"""ctypes binding of ``libtartarus.so`` (argument marshalling only).

The functions carry the names of the C ABI in ``include/tartarus.h``; every
step of the ray-tracing path runs in the library's HIP kernels.  torch supplies
device memory (output buffers, tables) and streams.  torch is imported before
the library is loaded so that both use the same HIP runtime.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os

import torch  # noqa: F401  (loads the HIP runtime the library shares)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtartarus.so")

OK, E_INVALID, E_NOMEM, E_DEVICE, E_TOO_LARGE, E_NOT_FOUND, E_AGAIN = 0, -1, -2, -3, -4, -5, -6
ESCAPED, CAPTURED, FAILED, ON_DISK = 0, 1, 2, 3
SHADE_OBSERVED, SHADE_INTRINSIC = 0, 1
SERVE_SMALLEST_FIRST, SERVE_ARRIVAL = 0, 1
METRIC_KERR, METRIC_TABLE = 0, 1
PREC_FP64, PREC_MIXED = 0, 1
ORDER_DEFAULT, ORDER_PIXEL, ORDER_COST, ORDER_TILE = 0, 1, 2, 3
METHOD_DP45, METHOD_CK45, METHOD_RKF45, METHOD_GBS, METHOD_VERLET = 0, 1, 2, 3, 4


class TartarusError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"tartarus error {code}: {msg}")
        self.code = code


class Metric(C.Structure):
    _fields_ = [("kind", C.c_int), ("a", C.c_double), ("table", C.c_void_p), ("nr", C.c_int),
                ("nth", C.c_int), ("r_min", C.c_double), ("r_max", C.c_double)]


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
                ("max_steps", C.c_int64), ("precision", C.c_int), ("method", C.c_int)]


OUTPUT_FIELDS = ("cls", "n_hits", "final_rtp", "h_drift", "h_gate", "hit_r", "hit_g", "hit_flux",
                 "hit_lambda", "hit_order", "intensity", "n_accept", "n_reject", "n_fp32", "n_cross")


class Outputs(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in OUTPUT_FIELDS]


class Launch(C.Structure):
    _fields_ = [("block_threads", C.c_int), ("blocks_per_cu", C.c_int), ("chunk", C.c_int),
                ("refill_min", C.c_int), ("order", C.c_int)]


_lib = None


def lib():
    """Load the built library; fail loudly if it is missing (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                               "or python paper_2609_08989_amd/build.py")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        L.tartarus_init.argtypes = [C.c_int, C.c_size_t]
        L.tartarus_shutdown.argtypes = []
        L.tartarus_validate.argtypes = [P(Metric), P(Camera), C.c_int, P(Disk), P(Solver)]
        L.tartarus_trace.argtypes = [P(Metric), P(Camera), C.c_int, P(Disk), P(Solver), P(Outputs), C.c_void_p]
        L.tartarus_trace_launch.argtypes = [P(Metric), P(Camera), C.c_int, P(Disk), P(Solver), P(Outputs),
                                            P(Launch), C.c_void_p]
        L.tartarus_trace_noalloc.argtypes = [P(Metric), P(Camera), C.c_int, P(Disk), P(Solver), P(Outputs),
                                             P(Launch), C.c_void_p]
        L.tartarus_autotune.argtypes = [P(Metric), P(Camera), C.c_int, P(Disk), P(Solver), P(Outputs),
                                        C.c_void_p, P(Launch)]
        L.tartarus_build_kerr_table.argtypes = [C.c_double, C.c_int, C.c_int, C.c_double, C.c_double,
                                                C.c_void_p, C.c_void_p]
        L.tartarus_submit.argtypes = [P(Metric), P(Camera), P(Disk), P(Solver), P(Outputs), P(C.c_uint64)]
        L.tartarus_poll.argtypes = [C.c_uint64, P(C.c_int)]
        L.tartarus_wait.argtypes = [C.c_uint64, C.c_int64]
        L.tartarus_serving_order.argtypes = [C.c_int]
        L.tartarus_kernel_timing.argtypes = [C.c_int]
        L.tartarus_kernel_time.argtypes = [P(C.c_double), P(C.c_longlong)]
        L.tartarus_cancel.argtypes = [C.c_uint64]
        L.tartarus_ticket_times.argtypes = [C.c_uint64, P(C.c_int64)]
        L.tartarus_last_error.restype = C.c_char_p
        L.tartarus_last_error.argtypes = []
        _lib = L
        # the serving thread must be stopped while the HIP runtime is still up
        atexit.register(L.tartarus_shutdown)
    return _lib


def _check(rc: int) -> int:
    if rc != OK:
        msg = lib().tartarus_last_error()
        raise TartarusError(rc, msg.decode() if msg else "")
    return rc


def _stream(stream) -> C.c_void_p:
    if stream is None:
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


# ---------------------------------------------------------------- struct builders
def make_metric(a: float, table: torch.Tensor | None = None, nr=0, nth=0, r_min=0.0, r_max=0.0) -> Metric:
    m = Metric(METRIC_KERR if table is None else METRIC_TABLE, float(a), None, 0, 0, 0.0, 0.0)
    if table is not None:
        m.table = C.c_void_p(table.data_ptr())
        m.nr, m.nth, m.r_min, m.r_max = int(nr), int(nth), float(r_min), float(r_max)
    return m


def make_camera(c: dict) -> Camera:
    return Camera(c["r_obs"], c["theta_obs"], c["nx"], c["ny"], c["alpha_min"], c["alpha_max"],
                  c["beta_min"], c["beta_max"])


def make_disk(d: dict | None) -> Disk:
    if d is None:
        return Disk(0.0, 0.0, 0, 0, 0)
    return Disk(d.get("r_in", 0.0), d["r_out"], d.get("max_hits", 3), d.get("opaque", 0), d.get("shading", 0))


def make_solver(s: dict, precision: int = PREC_FP64) -> Solver:
    return Solver(s["rtol"], s["atol"], s.get("h0_frac", 0.01), s.get("horizon_factor", 1.01),
                  s["r_escape"], s.get("event_tol", 1e-12), s.get("max_steps", 1_000_000), precision, s.get("method", 0))


def make_launch(block_threads=0, blocks_per_cu=0, chunk=0, refill_min=0, order=0) -> Launch:
    return Launch(block_threads, blocks_per_cu, chunk, refill_min, order)


def alloc_outputs(n: int, device="cuda") -> dict:
    """Caller-owned device output buffers for n rays (torch tensors)."""
    f64, i32 = torch.float64, torch.int32
    z = lambda *shape, dt: torch.zeros(*shape, dtype=dt, device=device)
    return {
        "cls": z(n, dt=i32), "n_hits": z(n, dt=i32), "final_rtp": z(n, 3, dt=f64), "h_drift": z(n, dt=f64),
        "h_gate": z(n, dt=f64), "hit_r": z(n, 3, dt=f64), "hit_g": z(n, 3, dt=f64), "hit_flux": z(n, 3, dt=f64),
        "hit_lambda": z(n, 3, dt=f64), "hit_order": z(n, 3, dt=i32), "intensity": z(n, dt=f64),
        "n_accept": z(n, dt=i32), "n_reject": z(n, dt=i32), "n_fp32": z(n, dt=i32), "n_cross": z(n, dt=i32),
    }


def outputs_struct(o: dict) -> Outputs:
    return Outputs(*[C.c_void_p(o[f].data_ptr()) for f in OUTPUT_FIELDS])


def to_numpy(o: dict) -> dict:
    return {k: v.cpu().numpy() for k, v in o.items()}


# ---------------------------------------------------------------- the C ABI
def tartarus_init(device: int = 0, hbm_budget_bytes: int = 0) -> None:
    _check(lib().tartarus_init(device, hbm_budget_bytes))


def tartarus_shutdown() -> None:
    _check(lib().tartarus_shutdown())


def tartarus_validate(metric: Metric, cams, disk: Disk, solver: Solver) -> int:
    cams = list(cams) if not isinstance(cams, Camera) else [cams]
    arr = (Camera * len(cams))(*cams)
    return lib().tartarus_validate(C.byref(metric), arr, len(cams), C.byref(disk), C.byref(solver))


def tartarus_trace(metric: Metric, cams, disk: Disk, solver: Solver, outputs: dict, stream=None,
                   launch: Launch | None = None) -> None:
    cams = list(cams) if not isinstance(cams, Camera) else [cams]
    arr = (Camera * len(cams))(*cams)
    so = outputs_struct(outputs)
    if launch is None:
        _check(lib().tartarus_trace(C.byref(metric), arr, len(cams), C.byref(disk), C.byref(solver),
                                    C.byref(so), _stream(stream)))
    else:
        _check(lib().tartarus_trace_launch(C.byref(metric), arr, len(cams), C.byref(disk), C.byref(solver),
                                           C.byref(so), C.byref(launch), _stream(stream)))


def tartarus_trace_noalloc(metric: Metric, cams, disk: Disk, solver: Solver, outputs: dict, stream=None,
                           launch: Launch | None = None) -> None:
    cams = list(cams) if not isinstance(cams, Camera) else [cams]
    arr = (Camera * len(cams))(*cams)
    so = outputs_struct(outputs)
    _check(lib().tartarus_trace_noalloc(C.byref(metric), arr, len(cams), C.byref(disk), C.byref(solver),
                                        C.byref(so), C.byref(launch) if launch is not None else None,
                                        _stream(stream)))


NOALLOC_MAX_RAYS, NOALLOC_MAX_CAMERAS = 262144, 64


def tartarus_autotune(metric: Metric, cams, disk: Disk, solver: Solver, outputs: dict, stream=None) -> Launch:
    cams = list(cams) if not isinstance(cams, Camera) else [cams]
    arr = (Camera * len(cams))(*cams)
    best = Launch()
    _check(lib().tartarus_autotune(C.byref(metric), arr, len(cams), C.byref(disk), C.byref(solver),
                                   C.byref(outputs_struct(outputs)), _stream(stream), C.byref(best)))
    return best


def tartarus_build_kerr_table(a: float, nr: int, nth: int, r_min: float, r_max: float, table: torch.Tensor,
                              stream=None) -> None:
    assert table.dtype == torch.float64 and table.is_cuda and table.numel() == nr * nth * 20
    _check(lib().tartarus_build_kerr_table(a, nr, nth, r_min, r_max, C.c_void_p(table.data_ptr()),
                                           _stream(stream)))


def tartarus_serving_order(order: int) -> None:
    _check(lib().tartarus_serving_order(int(order)))


def tartarus_kernel_timing(enable: bool) -> None:
    _check(lib().tartarus_kernel_timing(1 if enable else 0))


def tartarus_kernel_time() -> tuple:
    """(total milliseconds, launches) of the integrator launches timed since
    the last call."""
    ms, n = C.c_double(0.0), C.c_longlong(0)
    _check(lib().tartarus_kernel_time(C.byref(ms), C.byref(n)))
    return ms.value, n.value


def tartarus_submit(metric: Metric, cam: Camera, disk: Disk, solver: Solver, outputs: dict) -> int:
    t = C.c_uint64(0)
    _check(lib().tartarus_submit(C.byref(metric), C.byref(cam), C.byref(disk), C.byref(solver),
                                 C.byref(outputs_struct(outputs)), C.byref(t)))
    return t.value


def tartarus_poll(ticket: int) -> int:
    st = C.c_int(0)
    _check(lib().tartarus_poll(ticket, C.byref(st)))
    return st.value


def tartarus_wait(ticket: int, timeout_ms: int = -1) -> None:
    _check(lib().tartarus_wait(ticket, timeout_ms))


def tartarus_cancel(ticket: int) -> None:
    _check(lib().tartarus_cancel(ticket))


def tartarus_ticket_times(ticket: int):
    st = (C.c_int64 * 3)()
    _check(lib().tartarus_ticket_times(ticket, st))
    return list(st)


def tartarus_last_error() -> str:
    m = lib().tartarus_last_error()
    return m.decode() if m else ""
