"""C-ABI checks that need no GPU: the library loads, exports every function
declared in include/tartarus.h, and rejects invalid arguments before touching
the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "tartarus.h")


@pytest.fixture(scope="module")
def T():
    from paper_2609_08989_amd import build as b
    if not os.path.exists(b.LIB):
        b.build()
    from paper_2609_08989_amd import tartarus as T
    T.lib()
    return T


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(tartarus_\w+)\s*\(", text, flags=re.M)))


def test_every_declared_symbol_is_exported(T):
    names = declared_functions()
    assert len(names) >= 13
    raw = C.CDLL(T.LIB_PATH)
    missing = [n for n in names if not hasattr(raw, n)]
    assert not missing, missing


def good():
    import workloads as W
    from paper_2609_08989_amd import tartarus as T
    w = W.WORKLOADS["kerr09_512"]
    return (T.make_metric(0.9), T.make_camera(w["cameras"][0]), T.make_disk(w["disk"]),
            T.make_solver(w["solver"]))


def test_validate_accepts_the_workloads(T):
    m, c, d, s = good()
    assert T.tartarus_validate(m, c, d, s) == T.OK


@pytest.mark.parametrize("mutate,field", [
    (lambda m, c, d, s: setattr(m, "a", 1.0), "spin"),
    (lambda m, c, d, s: setattr(m, "a", -0.1), "spin"),
    (lambda m, c, d, s: setattr(c, "theta_obs", 0.0), "theta_obs"),
    (lambda m, c, d, s: setattr(c, "theta_obs", 3.2), "theta_obs"),
    (lambda m, c, d, s: setattr(c, "nx", 0), "nx"),
    (lambda m, c, d, s: setattr(c, "alpha_max", 2000.0), "window"),
    (lambda m, c, d, s: setattr(s, "rtol", 0.0), "rtol"),
    (lambda m, c, d, s: setattr(s, "atol", 0.0), "atol"),
    (lambda m, c, d, s: setattr(s, "r_escape", 900.0), "r_escape"),
    (lambda m, c, d, s: setattr(s, "r_escape", 2e15), "r_escape"),
    (lambda m, c, d, s: setattr(s, "horizon_factor", 0.9), "horizon_factor"),
    (lambda m, c, d, s: setattr(s, "max_steps", 0), "max_steps"),
    (lambda m, c, d, s: setattr(s, "precision", 5), "precision"),
    (lambda m, c, d, s: setattr(s, "method", 5), "method"),
    (lambda m, c, d, s: setattr(s, "method", -1), "method"),
    (lambda m, c, d, s: (setattr(s, "method", 1), setattr(s, "precision", 1)), "mixed needs DP45"),
    (lambda m, c, d, s: (setattr(s, "method", 3), setattr(s, "precision", 1)), "mixed needs DP45"),
    (lambda m, c, d, s: (setattr(s, "method", 4), setattr(s, "precision", 1)), "mixed needs DP45"),
    (lambda m, c, d, s: setattr(d, "max_hits", 4), "max_hits"),
    (lambda m, c, d, s: setattr(d, "opaque", 2), "opaque"),
    (lambda m, c, d, s: (setattr(d, "opaque", 1), setattr(d, "max_hits", 0)), "opaque needs a hit"),
    (lambda m, c, d, s: setattr(d, "shading", 2), "shading"),
    (lambda m, c, d, s: setattr(m, "kind", 7), "kind"),
])
def test_validate_rejects(T, mutate, field):
    m, c, d, s = good()
    mutate(m, c, d, s)
    assert T.tartarus_validate(m, c, d, s) == T.E_INVALID
    assert T.tartarus_last_error(), field


def test_table_metric_rules(T):
    m, c, d, s = good()
    m.kind = T.METRIC_TABLE
    assert T.tartarus_validate(m, c, d, s) == T.E_INVALID  # no table pointer
    m.table = C.c_void_p(0x1000)
    m.nr, m.nth, m.r_min, m.r_max = 512, 256, 1.9, 2000.0
    assert T.tartarus_validate(m, c, d, s) == T.OK
    for method in (T.METHOD_CK45, T.METHOD_GBS, T.METHOD_VERLET):
        s.method = method
        assert T.tartarus_validate(m, c, d, s) == T.E_INVALID  # tabulated metric: DP45 only
    s.method = T.METHOD_DP45
    s.precision = T.PREC_MIXED
    assert T.tartarus_validate(m, c, d, s) == T.E_INVALID  # tables are FP64 only
    s.precision = T.PREC_FP64
    # serving takes analytic Kerr requests only; the refusal needs no device
    fake = {f: type("P", (), {"data_ptr": lambda self: 0x1000})() for f in T.OUTPUT_FIELDS}
    so, t = T.outputs_struct(fake), C.c_uint64(0)
    assert T.lib().tartarus_submit(C.byref(m), C.byref(c), C.byref(d), C.byref(s), C.byref(so),
                                   C.byref(t)) == T.E_INVALID
    m.r_max = 1.0
    assert T.tartarus_validate(m, c, d, s) == T.E_INVALID


def test_six_stage_pairs_and_extrapolation_are_accepted(T):
    m, c, d, s = good()
    for method in (T.METHOD_CK45, T.METHOD_RKF45, T.METHOD_GBS, T.METHOD_VERLET):
        s.method = method
        assert T.tartarus_validate(m, c, d, s) == T.OK


def test_cameras_must_share_grid(T):
    m, c, d, s = good()
    c2 = T.Camera.from_buffer_copy(c)
    c2.nx = c.nx - 1
    assert T.tartarus_validate(m, [c, c2], d, s) == T.E_INVALID


def test_calls_before_init_fail_cleanly(T):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present; covered by the GPU tests")
    m, c, d, s = good()
    fake = {f: type("P", (), {"data_ptr": lambda self: 0x1000})() for f in T.OUTPUT_FIELDS}
    so = T.outputs_struct(fake)
    arr = (T.Camera * 1)(c)
    rc = T.lib().tartarus_trace(C.byref(m), arr, 1, C.byref(d), C.byref(s), C.byref(so), None)
    assert rc == T.E_DEVICE
    assert T.lib().tartarus_init(0, 0) == T.E_DEVICE
    st = C.c_int(0)
    assert T.lib().tartarus_poll(C.c_uint64(12345), C.byref(st)) == T.E_NOT_FOUND
    t = C.c_uint64(0)
    assert T.lib().tartarus_submit(C.byref(m), C.byref(c), C.byref(d), C.byref(s), C.byref(so), C.byref(t)) == T.E_DEVICE
    assert T.lib().tartarus_serving_order(T.SERVE_ARRIVAL) == T.E_DEVICE
    assert T.lib().tartarus_serving_order(7) == T.E_INVALID
    assert T.lib().tartarus_kernel_timing(1) == T.E_DEVICE
    assert T.lib().tartarus_kernel_timing(2) == T.E_INVALID
    ms, n = C.c_double(0.0), C.c_longlong(0)
    assert T.lib().tartarus_kernel_time(C.byref(ms), C.byref(n)) == T.E_DEVICE
    assert T.lib().tartarus_kernel_time(None, C.byref(n)) == T.E_INVALID


def test_null_outputs_rejected(T):
    m, c, d, s = good()
    arr = (T.Camera * 1)(c)
    assert T.lib().tartarus_trace(C.byref(m), arr, 1, C.byref(d), C.byref(s), None, None) == T.E_INVALID


def test_noalloc_argument_errors_need_no_device(T):
    """The allocation-free trace checks its limits before any device work: the
    tabulated metric and over-size requests are refused with the right status."""
    import workloads as W
    w = W.WORKLOADS["kerr09_512"]
    fake = T.Outputs(*([C.c_void_p(0x1000)] * len(T.OUTPUT_FIELDS)))
    L = T.lib()
    cam = T.make_camera(dict(w["cameras"][0], nx=513, ny=512))
    args = (C.byref(T.make_metric(0.9)), (T.Camera * 1)(cam), 1, C.byref(T.make_disk(w["disk"])),
            C.byref(T.make_solver(w["solver"])), C.byref(fake), None, None)
    assert L.tartarus_trace_noalloc(*args) == T.E_TOO_LARGE
    cams = (T.Camera * 65)(*([T.make_camera(dict(w["cameras"][0], nx=4, ny=4))] * 65))
    assert L.tartarus_trace_noalloc(C.byref(T.make_metric(0.9)), cams, 65, C.byref(T.make_disk(w["disk"])),
                                    C.byref(T.make_solver(w["solver"])), C.byref(fake), None, None) == T.E_TOO_LARGE
    tab = T.Metric(T.METRIC_TABLE, 0.7, C.c_void_p(0x1000), 64, 32, 1.9, 2000.0)
    small = (T.Camera * 1)(T.make_camera(dict(w["cameras"][0], nx=8, ny=8)))
    assert L.tartarus_trace_noalloc(C.byref(tab), small, 1, C.byref(T.make_disk(w["disk"])),
                                    C.byref(T.make_solver(w["solver"])), C.byref(fake), None, None) == T.E_INVALID
    assert "analytic Kerr" in T.tartarus_last_error()
