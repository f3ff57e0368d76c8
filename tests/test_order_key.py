"""Scheduling key of the cost-ordered queue (csrc/order.hpp), built for the host
with g++: rays on the critical curve of Kerr (the spherical photon orbits,
Bardeen's parametrisation) fall in the top bucket, and the key falls off with
the distance from that curve.  The key never enters a ray's arithmetic; GPU
tests check that traced results do not depend on the queue order."""
import ctypes as C
import os
import subprocess
import tempfile

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = r"""
#include "order.hpp"
extern "C" void run(double a, const double* b, const double* q, int* k, double* d, long n) {
    const double rp = 1.0 + __builtin_sqrt(1.0 - a * a);
    for (long i = 0; i < n; ++i) {
        k[i] = tartarus::cost_bucket(a, b[i], q[i], rp);
        d[i] = tartarus::critical_distance(a, b[i], q[i], rp);
    }
}
"""


@pytest.fixture(scope="module")
def lib():
    d = tempfile.mkdtemp()
    src, so = os.path.join(d, "t.cpp"), os.path.join(d, "t.so")
    open(src, "w").write(SRC)
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                    "-I", os.path.join(ROOT, "paper_2609_08989_amd", "csrc"), src, "-o", so], check=True)
    L = C.CDLL(so)
    dp = C.POINTER(C.c_double)
    L.run.argtypes = [C.c_double, dp, dp, C.POINTER(C.c_int), dp, C.c_long]
    return L


def run(L, a, b, q):
    b = np.ascontiguousarray(b, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    k = np.zeros(len(b), dtype=np.int32)
    d = np.zeros(len(b))
    L.run(a, b.ctypes.data_as(C.POINTER(C.c_double)), q.ctypes.data_as(C.POINTER(C.c_double)),
          k.ctypes.data_as(C.POINTER(C.c_int)), d.ctypes.data_as(C.POINTER(C.c_double)), len(b))
    return k, d


def critical_curve(a, n=200):
    """Constants (b, q) of the spherical photon orbits of Kerr (M = 1), radius
    between the prograde and retrograde circular photon orbits."""
    r1 = 2.0 * (1.0 + np.cos(2.0 / 3.0 * np.arccos(-a)))
    r2 = 2.0 * (1.0 + np.cos(2.0 / 3.0 * np.arccos(a)))
    r = np.linspace(r1, r2, n + 2)[1:-1]
    b = -(r**3 - 3 * r**2 + a * a * r + a * a) / (a * (r - 1.0))
    q = -r**3 * (r**3 - 6 * r**2 + 9 * r - 4 * a * a) / (a * a * (r - 1.0) ** 2)
    return b, q


def test_schwarzschild_critical_circle_is_top_bucket(lib):
    # a = 0: the critical curve is b^2 + q = 27
    phi = np.linspace(0.01, np.pi - 0.01, 101)
    b = np.sqrt(27.0) * np.cos(phi)
    q = 27.0 - b * b
    k, d = run(lib, 0.0, b, q)
    assert np.abs(d).max() < 1e-12
    assert (k == 31).all()


@pytest.mark.parametrize("a", [0.3, 0.9, 0.998])
def test_kerr_critical_curve_is_top_bucket(lib, a):
    b, q = critical_curve(a)
    k, d = run(lib, a, b, q)
    assert np.abs(d).max() < 1e-9
    assert (k >= 30).all()


@pytest.mark.parametrize("a", [0.0, 0.9])
def test_key_falls_off_with_distance(lib, a):
    if a == 0.0:
        b = np.array([2.0, -3.0, 4.5])
        q = 27.0 - b * b
    else:
        b, q = critical_curve(a, 5)
    for sign in (+1.0, -1.0):          # captured side and escaping side of the curve
        eps = (1e-6, 1e-4, 1e-1, 1.0, 10.0)
        res = [run(lib, a, b, q + sign * e) for e in eps]
        # |D| grows linearly with the offset near the curve (a simple double root splits)
        ratio = np.abs(res[1][1]) / np.abs(res[0][1])
        assert ((ratio > 50) & (ratio < 200)).all()
        keys = [k for k, _ in res]
        for near, far in zip(keys, keys[1:]):
            assert (far <= near).all()
        assert (keys[-1] < keys[0]).all()
    # far from the curve: low buckets
    k, _ = run(lib, a, np.array([0.0, 20.0, -20.0]), np.array([200.0, 10.0, 10.0]))
    assert (k <= 14).all()
