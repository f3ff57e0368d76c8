"""The integrator's compact FP64 sine/cosine (csrc/fastmath.hpp), built for the
host with g++ and compared with the C library's sin and cos: within 2 ulp on
the polar-angle range a ray visits, and on quadrant boundaries."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = r"""
#include "fastmath.hpp"
extern "C" void run(const double* x, double* s, double* c, long n) {
    for (long i = 0; i < n; ++i) tartarus::sincos64(x[i], s + i, c + i);
}
extern "C" void run32(const float* x, float* s, float* c, long n) {
    for (long i = 0; i < n; ++i) tartarus::sincos32(x[i], s + i, c + i);
}
extern "C" void shift(const double* s0, const double* c0, const double* dt, double* s, double* c, long n) {
    for (long i = 0; i < n; ++i) tartarus::sincos_shift(s0[i], c0[i], dt[i], s[i], c[i], tartarus::ShiftImm{});
}
"""


@pytest.fixture(scope="module")
def lib():
    d = tempfile.mkdtemp()
    src = os.path.join(d, "t.cpp")
    so = os.path.join(d, "t.so")
    open(src, "w").write(SRC)
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-shared", "-fPIC",
                    "-I", os.path.join(ROOT, "paper_2609_08989_amd", "csrc"), src, "-o", so], check=True)
    L = C.CDLL(so)
    dp = C.POINTER(C.c_double)
    L.run.argtypes = [dp, dp, dp, C.c_long]
    fp = C.POINTER(C.c_float)
    L.run32.argtypes = [fp, fp, fp, C.c_long]
    L.shift.argtypes = [dp, dp, dp, dp, dp, C.c_long]
    return L


def run(L, x):
    x = np.ascontiguousarray(x, dtype=np.float64)
    s, c = np.zeros_like(x), np.zeros_like(x)
    p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    L.run(p(x), p(s), p(c), len(x))
    return s, c


def test_sincos_accuracy(lib):
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.uniform(-10, 10, 200000), np.linspace(-7, 7, 20001),
                        np.pi / 2 * np.arange(-8, 9), np.pi / 2 * np.arange(-8, 9) + 1e-9,
                        np.array([0.0, 1e-300, -1e-20, 0.5, 1.0, 3.0])])
    s, c = run(lib, x)
    es, ec = np.sin(x), np.cos(x)
    # error in units of the last place of the magnitude (1 ulp of 1.0 = 2.2e-16)
    ulp_s = np.abs(s - es) / np.spacing(np.maximum(np.abs(es), 1e-300))
    ulp_c = np.abs(c - ec) / np.spacing(np.maximum(np.abs(ec), 1e-300))
    big_s, big_c = np.abs(es) > 1e-3, np.abs(ec) > 1e-3
    assert ulp_s[big_s].max() <= 2.0 and ulp_c[big_c].max() <= 2.0
    # near the zeros: absolute error well below an ulp of 1
    assert np.abs(s - es).max() < 2.3e-16 and np.abs(c - ec).max() < 2.3e-16


def test_equator_sign(lib):
    # the disk event tests the sign of cos(theta) next to pi/2
    x = np.nextafter(np.pi / 2, 0) - np.arange(0, 50) * 1e-16
    s, c = run(lib, x)
    assert np.all(c > 0)
    x = np.pi / 2 + 1e-15 + np.arange(0, 50) * 1e-16
    s, c = run(lib, x)
    assert np.all(c < 0)


def test_sincos32_accuracy(lib):
    """Single-precision sin/cos of the FP32 far-field stages: within 2 ulp of
    float for |sin|, |cos| > 1e-3 (absolute 1.2e-7 near the zeros)."""
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-10, 10, 200000), np.linspace(-7, 7, 20001)]).astype(np.float32)
    s, c = np.zeros_like(x), np.zeros_like(x)
    fp = lambda a: a.ctypes.data_as(C.POINTER(C.c_float))
    lib.run32(fp(x), fp(s), fp(c), len(x))
    xd = x.astype(np.float64)
    es, ec = np.sin(xd), np.cos(xd)
    us = np.abs(s - es) / np.spacing(np.maximum(np.abs(es), 1e-30).astype(np.float32))
    uc = np.abs(c - ec) / np.spacing(np.maximum(np.abs(ec), 1e-30).astype(np.float32))
    assert us[np.abs(es) > 1e-3].max() <= 2.0 and uc[np.abs(ec) > 1e-3].max() <= 2.0
    assert np.abs(s - es).max() < 1.2e-7 and np.abs(c - ec).max() < 1.2e-7


def test_sincos_wide_arguments_and_quadrants(lib):
    """Up to the documented |x| < 1e6 (quadrant index k up to ~6.4e5): the
    three-part reduction and the 32-bit quadrant keep 2 ulp for |sin|, |cos| >
    1e-3, every quadrant of negative and positive k included."""
    rng = np.random.default_rng(2)
    x = np.concatenate([rng.uniform(-1e6, 1e6, 100000), rng.uniform(-1e3, 1e3, 100000),
                        np.pi / 2 * np.arange(-40, 41) + 0.3])
    s, c = run(lib, x)
    es, ec = np.sin(x), np.cos(x)
    us = np.abs(s - es) / np.spacing(np.abs(es))
    uc = np.abs(c - ec) / np.spacing(np.abs(ec))
    assert us[np.abs(es) > 1e-3].max() <= 2.0 and uc[np.abs(ec) > 1e-3].max() <= 2.0
    # every quadrant q = k mod 4 of both signs of k is exercised above
    k = np.rint(x * (2 / np.pi)).astype(np.int64)
    assert set((k[k < 0] % 4).tolist()) == {0, 1, 2, 3} and set((k[k > 0] % 4).tolist()) == {0, 1, 2, 3}
    s0, c0 = run(lib, np.array([0.0, -0.0]))
    assert np.all(s0 == 0.0) and np.all(c0 == 1.0)


def test_angle_shift_accuracy(lib):
    """sin and cos of theta0 + d from those of theta0 (the integrator's stages
    near the step's start), for |d| <= 1/16 and |d| <= |sin(theta0)| / 2, the
    bounds the kernel applies, given correctly rounded sin and cos of theta0;
    theta0 + d is exact, as the stage angle minus the step's start is in the
    kernel.  Against the C library: within 2 ulp where |sin|, |cos| >= 0.1;
    the sine within 3 ulp relative next to both poles (where 1/sin^2 enters the
    right-hand side); everywhere within one ulp of 1 absolute, which near the
    equator is the cosine's own uncertainty from rounding theta (ulp(pi/2))."""
    rng = np.random.default_rng(3)
    n = 200000
    th = np.concatenate([rng.uniform(0.002, np.pi - 0.002, n), rng.uniform(-0.5, 3.6, n // 4),
                         rng.uniform(0.0005, 0.05, n // 8), np.pi - rng.uniform(0.0005, 0.05, n // 8),
                         np.array([np.pi / 2, np.pi / 2 + 1e-12, 0.05, np.pi - 0.05])])
    lim = np.minimum(1.0 / 16.0, 0.5 * np.abs(np.sin(th)))
    d = rng.uniform(-1.0, 1.0, th.size) * lim
    d[-4:] = [1.0 / 16.0, -1.0 / 16.0, 0.025, -0.025]
    th1 = th + d
    d = th1 - th                  # exact: the shifted angle is th1 itself
    s0, c0 = np.sin(th), np.cos(th)
    s, c = np.zeros_like(th), np.zeros_like(th)
    p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    lib.shift(p(s0), p(c0), p(d), p(s), p(c), th.size)
    es, ec = np.sin(th1), np.cos(th1)
    us = np.abs(s - es) / np.spacing(np.abs(es))
    uc = np.abs(c - ec) / np.spacing(np.abs(ec))
    assert us[np.abs(es) >= 0.1].max() <= 2.0 and uc[np.abs(ec) >= 0.1].max() <= 2.0
    assert np.abs(s - es).max() < 2.3e-16 and np.abs(c - ec).max() < 2.3e-16
    poles = ((np.abs(th1) < 0.05) | (np.abs(th1 - np.pi) < 0.05)) & (es != 0.0)
    assert poles.sum() > 10000 and us[poles].max() <= 3.0
    # beyond its bound the shift is not used: at |d| = 1/4 its error is far above an ulp
    s2, c2 = np.zeros(1), np.zeros(1)
    t0 = np.array([1.0])
    dd = np.array([0.25])
    lib.shift(p(np.sin(t0)), p(np.cos(t0)), p(dd), p(s2), p(c2), 1)
    assert abs(s2[0] - np.sin(1.25)) > 1e-14
