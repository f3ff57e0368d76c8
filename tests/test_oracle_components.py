"""Pins of the oracle's camera, integrator pieces and emitter model (CPU only).

* Camera (Sec. 2.2): the null condition of Eq. (4)-(5) (the paper states the
  projection makes H = 0), the ZAMO frame rebuilt independently as the unit
  normal of t = const, and the exact Schwarzschild impact parameter.
* Dormand-Prince 5(4) (Sec. 3.2): exact order conditions of the published
  tableau, observed order 5 and the h^5 embedded error on a test ODE.
* Dense output / events: the cubic Hermite interpolant is exact on cubics;
  the bisection count is the smallest n with h / 2^n <= tol.
* Emitter (Secs. 2.3-2.4): ISCO as the minimum of the circular-orbit energy,
  Eq. (11) against the Page-Thorne integral definition, Eq. (15) against the
  textbook circular-orbit u^t.
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.optimize import minimize_scalar

import workloads as W


def cam(r_obs, th_deg, nx, ny, w):
    return W.camera(r_obs, th_deg, nx, ny, w)


CAMS = [(0.0, cam(1000.0, 90.0, 9, 7, 10.0)), (0.9, cam(1000.0, 60.0, 9, 7, 25.0)),
        (0.998, cam(1000.0, 17.0, 6, 6, 20.0)), (0.5, cam(100.0, 85.0, 5, 5, 20.0))]


# ----------------------------------------------------------------- camera
@pytest.mark.parametrize("a,c", CAMS)
def test_initial_state_is_null(orc, a, c):
    m = orc.make_metric(a)
    ca = orc.make_camera(c)
    for j in range(c["ny"]):
        for i in range(c["nx"]):
            q = orc.initial_state(m, ca, i, j)
            assert abs(orc.hamiltonian(m, q)) < 2e-15
            assert orc.rhs(m, q)[1] < 0.0  # traced backward: moves inward first


@pytest.mark.parametrize("a,c", CAMS)
def test_local_momentum_in_independent_zamo_frame(orc, a, c):
    """Project the photon momentum on a ZAMO frame built from the inverse metric
    (u^mu = -g^{mu t} / sqrt(-g^{tt}), the unit normal of t = const) and recover
    the local components of Eq. (4)."""
    m = orc.make_metric(a)
    ca = orc.make_camera(c)
    D, th = c["r_obs"], c["theta_obs"]
    g, _, _ = orc.metric_eval(m, D, th)
    G = np.zeros((4, 4))
    G[0, 0], G[0, 3], G[3, 0], G[1, 1], G[2, 2], G[3, 3] = g[0], g[1], g[1], g[2], g[3], g[4]
    Gi = np.linalg.inv(G)
    u = -Gi[:, 0] / math.sqrt(-Gi[0, 0])
    assert u @ G @ u == pytest.approx(-1.0, rel=1e-13)
    for j in range(c["ny"]):
        for i in range(c["nx"]):
            al = c["alpha_min"] + i * (c["alpha_max"] - c["alpha_min"]) / (c["nx"] - 1)
            be = c["beta_min"] + j * (c["beta_max"] - c["beta_min"]) / (c["ny"] - 1)
            q = orc.initial_state(m, ca, i, j)
            p = -q[4:]  # undo the backward-tracing sign flip
            local = np.array([-(p @ u), p[1] / math.sqrt(g[2]), p[2] / math.sqrt(g[3]), p[3] / math.sqrt(g[4])])
            expect = np.array([1.0, math.sqrt(1 - (al * al + be * be) / D ** 2), be / D, -al / D])
            assert np.allclose(local, expect, rtol=1e-12, atol=1e-14)


def test_schwarzschild_impact_parameter_exact(orc):
    """a = 0, equatorial observer, beta = 0: b = L/E = |alpha| / sqrt(1 - 2/D)."""
    m = orc.make_metric(0.0)
    D = 1000.0
    c = cam(D, 90.0, 5, 1, 8.0)
    c["beta_min"] = c["beta_max"] = 0.0
    ca = orc.make_camera(c)
    for i in range(5):
        al = -8.0 + 4.0 * i
        q = orc.initial_state(m, ca, i, 0)
        E, L = q[4], -q[7]
        assert abs(L / E) == pytest.approx(abs(al) / math.sqrt(1 - 2 / D), rel=1e-14, abs=1e-14)
        assert q[6] == 0.0


def test_bardeen_mapping_at_finite_distance(orc):
    """Far from the hole the paper's (alpha, beta) equal Bardeen's celestial
    coordinates times sqrt(1 - 2/D) up to O(1/D) corrections (~1e-6 at D = 1000)."""
    a, iota, D = 0.9, 60.0 * math.pi / 180.0, 1000.0
    m = orc.make_metric(a)
    c = cam(D, 60.0, 7, 7, 25.0)
    ca = orc.make_camera(c)
    for j in range(7):
        for i in range(7):
            al = -25 + i * 50 / 6
            be = -25 + j * 50 / 6
            q = orc.initial_state(m, ca, i, j)
            E, L = q[4], -q[7]
            Q = q[6] ** 2 + math.cos(iota) ** 2 * (L * L / math.sin(iota) ** 2 - a * a * E * E)
            xi, eta = L / E, Q / E ** 2
            aB = -xi / math.sin(iota)
            bB = math.copysign(math.sqrt(max(0.0, eta + a * a * math.cos(iota) ** 2 - xi ** 2 / math.tan(iota) ** 2)), -q[6])
            s = math.sqrt(1 - 2 / D)
            assert aB * s == pytest.approx(al, abs=2e-5)
            assert bB * s == pytest.approx(be, abs=2e-5)


# ----------------------------------------------------------------- DP45
def as_fractions(x):
    out = []
    for v in np.ravel(x):
        f = Fraction(v).limit_denominator(10 ** 7)
        assert float(f) == v
        out.append(f)
    return np.array(out, dtype=object).reshape(np.shape(x))


def order_conditions(b, A, c):
    """Elementary weights of the 17 rooted trees up to order 5, with their densities."""
    n = len(b)
    Ac = [sum(A[i][j] * c[j] for j in range(n)) for i in range(n)]
    Ac2 = [sum(A[i][j] * c[j] ** 2 for j in range(n)) for i in range(n)]
    AAc = [sum(A[i][j] * Ac[j] for j in range(n)) for i in range(n)]
    Ac3 = [sum(A[i][j] * c[j] ** 3 for j in range(n)) for i in range(n)]
    AcAc = [sum(A[i][j] * c[j] * Ac[j] for j in range(n)) for i in range(n)]
    AAc2 = [sum(A[i][j] * Ac2[j] for j in range(n)) for i in range(n)]
    AAAc = [sum(A[i][j] * AAc[j] for j in range(n)) for i in range(n)]
    S = lambda v: sum(b[i] * v[i] for i in range(n))
    one = [Fraction(1)] * n
    conds = [
        (S(one), Fraction(1)),
        (S(c), Fraction(1, 2)),
        (S([x ** 2 for x in c]), Fraction(1, 3)), (S(Ac), Fraction(1, 6)),
        (S([x ** 3 for x in c]), Fraction(1, 4)), (S([c[i] * Ac[i] for i in range(n)]), Fraction(1, 8)),
        (S(Ac2), Fraction(1, 12)), (S(AAc), Fraction(1, 24)),
        (S([x ** 4 for x in c]), Fraction(1, 5)), (S([c[i] ** 2 * Ac[i] for i in range(n)]), Fraction(1, 10)),
        (S([c[i] * Ac2[i] for i in range(n)]), Fraction(1, 15)), (S([c[i] * AAc[i] for i in range(n)]), Fraction(1, 30)),
        (S([Ac[i] ** 2 for i in range(n)]), Fraction(1, 20)), (S(Ac3), Fraction(1, 20)),
        (S(AcAc), Fraction(1, 40)), (S(AAc2), Fraction(1, 60)), (S(AAAc), Fraction(1, 120)),
    ]
    return conds


@pytest.mark.parametrize("method", [0, 1, 2], ids=["dp45", "ck45", "rkf45"])
def test_rk_tableau_order_conditions(orc, method):
    """Each 5(4) pair of Sec. 3.2 (Dormand-Prince, Cash-Karp, Fehlberg): the
    propagating weights satisfy all 17 order conditions up to order 5, the
    embedded ones those up to order 4 and not all of order 5."""
    c, a6, b, bs = orc.rk_tableau(method)
    A = np.zeros((7, 7), dtype=object)
    A[:, :] = Fraction(0)
    A[:, :6] = as_fractions(a6)
    c = as_fractions(c)
    b = as_fractions(b)
    bs = as_fractions(bs)
    for i in range(7):
        assert sum(A[i]) == c[i]  # row sums give the nodes
    assert all(A[6][j] == b[j] for j in range(6)) and b[6] == 0  # first same as last
    full = order_conditions(list(b), A.tolist(), list(c))
    assert all(v == want for v, want in full)  # fifth order
    emb = order_conditions(list(bs), A.tolist(), list(c))
    assert all(v == want for v, want in emb[:8])  # embedded pair: fourth order
    assert any(v != want for v, want in emb[8:])  # ... and not fifth


@pytest.mark.parametrize("method", [0, 1, 2], ids=["dp45", "ck45", "rkf45"])
def test_rk_convergence_order_five(orc, method):
    f = lambda y: np.array([y[1], -y[0]])
    T = 2.0
    errs, ests = [], []
    for N in (10, 20, 40):
        y, e = orc.rk_fixed(method, f, [1.0, 0.0], T / N, N)
        errs.append(np.hypot(y[0] - math.cos(T), y[1] + math.sin(T)))
        ests.append(np.abs(e).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 24 < r1 < 44 and 24 < r2 < 44  # global error ~ h^5
    assert 24 < ests[0] / ests[1] < 44 and 24 < ests[1] / ests[2] < 44  # embedded estimate ~ h^5


# ------------------------------------------------- Gragg-Bulirsch-Stoer
@pytest.mark.parametrize("K", [2, 3, 4, 5, 6])
def test_gbs_exact_on_polynomials_of_degree_2k_minus_1(orc, K):
    """On y' = p(t) the smoothed modified midpoint rule is the composite trapezoid
    rule, whose error expands in even powers of the substep; K columns of
    extrapolation in h^2 remove K - 1 of those terms, so one macro-step is exact
    (to rounding) for deg p <= 2K - 1 and not for deg p = 2K."""
    rng = np.random.default_rng(K)
    t0, H = 0.3, 0.9
    for deg, exact_expected in ((2 * K - 1, True), (2 * K, False)):
        co = rng.normal(size=deg + 1)
        f = lambda y: np.array([1.0, np.polyval(co, y[0])])
        y, e = orc.gbs_fixed(K, f, [t0, 0.0], H, 1)
        P = np.polyint(co)
        exact = np.polyval(P, t0 + H) - np.polyval(P, t0)
        if exact_expected:
            assert abs(y[1] - exact) < 1e-13 * max(1.0, abs(exact))
        else:
            assert abs(y[1] - exact) > 1e-12
        assert y[0] == pytest.approx(t0 + H, abs=1e-13)


@pytest.mark.parametrize("K", [2, 3, 4])
def test_gbs_convergence_order_2k(orc, K):
    """The diagonal entry T[K][K] converges with order 2K; the error estimate
    T[K][K] - T[K][K-1] (the error of the order 2K - 2 entry) with order 2K - 1."""
    f = lambda y: np.array([y[1], -y[0]])
    T = 2.0
    errs, ests = [], []
    for N in (4, 8, 16):
        y, e = orc.gbs_fixed(K, f, [1.0, 0.0], T / N, N)
        errs.append(np.hypot(y[0] - math.cos(T), y[1] + math.sin(T)))
        ests.append(np.abs(e).max())
    want = 2.0 ** (2 * K)
    assert 0.85 * want < errs[0] / errs[1] < 1.15 * want
    assert 0.85 * want < errs[1] / errs[2] < 1.15 * want
    west = 2.0 ** (2 * K - 1)
    assert 0.7 * west < ests[1] / ests[2] < 1.3 * west


def test_gbs_columns_used_for_rays(orc):
    assert orc.gbs_columns() == 6


# ------------------------------------------------------------------ Verlet
def test_verlet_harmonic_oscillator_closed_form(orc):
    """On H = (p^2 + q^2)/2 the step is the linear map M = [[1 - h^2/2, h],
    [-h (1 - h^2/4), 1 - h^2/2]] (det 1, trace 2 - h^2), so N steps are
    M^N = U_{N-1}(c) M - U_{N-2}(c) I with c = cos(theta) = 1 - h^2/2 and the
    Chebyshev U_k = sin((k+1) theta) / sin(theta)."""
    h, N = 0.1, 1000
    y0 = np.array([1.0, 0.3])
    y, done = orc.verlet_fixed(lambda y: np.array([y[1], -y[0]]), y0, h, N)
    assert done == N
    th = math.acos(1 - h * h / 2)
    M = np.array([[1 - h * h / 2, h], [-h * (1 - h * h / 4), 1 - h * h / 2]])
    U = lambda k: math.sin((k + 1) * th) / math.sin(th)
    assert np.abs(y - (U(N - 1) * M - U(N - 2) * np.eye(2)) @ y0).max() < 1e-12


def nonseparable(y):
    """H = p^2 (1 + x^2) / 2 + x^2 / 2: kinetic and potential parts do not split."""
    return np.array([y[1] * (1 + y[0] ** 2), -(y[0] * y[1] ** 2 + y[0])])


def test_verlet_time_reversible_and_symplectic(orc):
    y0 = np.array([0.7, 0.4])
    yf, _ = orc.verlet_fixed(nonseparable, y0, 0.05, 2000)
    yb, done = orc.verlet_fixed(nonseparable, yf, -0.05, 2000)
    assert done == 2000
    assert np.abs(yb - y0).max() < 1e-11          # h -> -h retraces the path
    d, J = 1e-6, np.zeros((2, 2))
    for k in range(2):
        e = np.zeros(2)
        e[k] = d
        J[:, k] = (orc.verlet_fixed(nonseparable, y0 + e, 0.2, 1)[0]
                   - orc.verlet_fixed(nonseparable, y0 - e, 0.2, 1)[0]) / (2 * d)
    assert abs(np.linalg.det(J) - 1.0) < 1e-8    # area preserving (one degree of freedom)


def test_verlet_second_order_and_bounded_energy(orc):
    from scipy.integrate import solve_ivp
    y0, T = np.array([0.7, 0.4]), 3.0
    ref = solve_ivp(lambda t, y: nonseparable(y), (0, T), y0, method="DOP853", rtol=1e-13, atol=1e-14).y[:, -1]
    errs = [np.abs(orc.verlet_fixed(nonseparable, y0, T / n, n)[0] - ref).max() for n in (60, 120, 240)]
    assert 3.8 < errs[0] / errs[1] < 4.2 and 3.8 < errs[1] / errs[2] < 4.2
    H = lambda y: 0.5 * y[1] ** 2 * (1 + y[0] ** 2) + 0.5 * y[0] ** 2
    y, dev = y0.copy(), []
    for _ in range(1000):
        y, _ = orc.verlet_fixed(nonseparable, y, 0.1, 50)
        dev.append(abs(H(y) - H(y0)))
    dev = np.array(dev)
    assert dev[-100:].max() < 1.05 * dev[:100].max()   # no secular drift over 5e4 steps


# ----------------------------------------------------------------- events
def test_hermite_exact_on_cubics(orc):
    rng = np.random.default_rng(3)
    for _ in range(20):
        co = rng.normal(size=4)
        p = lambda x: co[0] + co[1] * x + co[2] * x ** 2 + co[3] * x ** 3
        dp = lambda x: co[1] + 2 * co[2] * x + 3 * co[3] * x ** 2
        x0, h = rng.normal(), abs(rng.normal()) + 0.1
        for s in (0.0, 0.2, 0.5, 0.77, 1.0):
            got = orc.hermite(s, p(x0), dp(x0), p(x0 + h), dp(x0 + h), h)
            assert got == pytest.approx(p(x0 + s * h), rel=1e-13, abs=1e-13)


def test_bisect_count_rule(orc):
    assert orc.bisect_count(1.0, 1e-12) == 40
    assert orc.bisect_count(1e-12, 1e-12) == 0
    assert orc.bisect_count(0.5e-12, 1e-12) == 0
    for h in (3.7, 120.0, 0.013):
        n = orc.bisect_count(h, 1e-12)
        assert h / 2 ** n <= 1e-12 < h / 2 ** (n - 1)


# ----------------------------------------------------------------- emitter
def circular_orbit(a, r):
    """Textbook prograde circular equatorial orbit in Kerr (Bardeen, Press & Teukolsky)."""
    den = r ** 0.75 * math.sqrt(r ** 1.5 - 3 * math.sqrt(r) + 2 * a)
    E = (r ** 1.5 - 2 * math.sqrt(r) + a) / den
    L = (r * r - 2 * a * math.sqrt(r) + a * a) / den
    Om = 1 / (r ** 1.5 + a)
    ut = (r ** 1.5 + a) / den
    return E, L, Om, ut


@pytest.mark.parametrize("a,ref", [(0.0, 6.0), (0.9, 2.3208830418), (0.998, 1.2369706552), (0.7, 3.3931284702)])
def test_isco(orc, a, ref):
    assert orc.isco(a) == pytest.approx(ref, rel=1e-10)
    # the ISCO is where the circular-orbit energy is minimal
    res = minimize_scalar(lambda r: circular_orbit(a, r)[0], bounds=(ref * 0.9, ref * 1.2), method="bounded",
                          options=dict(xatol=1e-10))
    assert res.x == pytest.approx(orc.isco(a), rel=2e-4)


def page_thorne_integral(a, r):
    """F = f / r with f = -Omega' (E - Omega L)^-2 int_{r_isco}^r (E - Omega L) L' dr (units Mdot/4pi)."""
    rin = orc_isco_cache[a]
    d = lambda fn, x, e=1e-6: (fn(x + e) - fn(x - e)) / (2 * e)
    E = lambda x: circular_orbit(a, x)[0]
    L = lambda x: circular_orbit(a, x)[1]
    Om = lambda x: circular_orbit(a, x)[2]
    I = quad(lambda x: (E(x) - Om(x) * L(x)) * d(L, x), rin, r, epsabs=1e-14, epsrel=1e-12, limit=200)[0]
    return -d(Om, r) / (E(r) - Om(r) * L(r)) ** 2 * I / r


orc_isco_cache = {}


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9, 0.998])
def test_flux_equals_page_thorne_integral(orc, a):
    rin = orc.isco(a)
    orc_isco_cache[a] = rin
    assert orc.nt_flux(a, rin, 50.0, rin) == 0.0
    assert orc.nt_flux(a, rin, 50.0, 0.99 * rin) == 0.0 and orc.nt_flux(a, rin, 50.0, 51.0) == 0.0
    for r in (1.05 * rin, 1.5 * rin, 10.0, 30.0):
        assert orc.nt_flux(a, rin, 50.0, r) == pytest.approx(page_thorne_integral(a, r), rel=1e-7)


@pytest.mark.parametrize("a,rpk", [(0.0, 9.550928), (0.9, 3.441843), (0.998, 1.581185)])
def test_flux_peak_radius(orc, a, rpk):
    rin = orc.isco(a)
    res = minimize_scalar(lambda r: -orc.nt_flux(a, rin, 100.0, r), bounds=(rin * 1.01, 20.0), method="bounded",
                          options=dict(xatol=1e-9))
    assert res.x == pytest.approx(rpk, rel=1e-5)


def test_flux_schwarzschild_classic_form(orc):
    rin = 6.0
    for r in (6.5, 9.0, 20.0, 80.0):
        x, s3 = math.sqrt(r), math.sqrt(3.0)
        classic = 3 / (2 * r ** 2.5 * (r - 3)) * (
            x - math.sqrt(6) - s3 / 2 * math.log((x - s3) / (math.sqrt(6) - s3))
            + s3 / 2 * math.log((x + s3) / (math.sqrt(6) + s3)))
        assert orc.nt_flux(0.0, rin, 100.0, r) == pytest.approx(classic, rel=1e-13)


@pytest.mark.parametrize("a", [0.0, 0.5, 0.9, 0.998])
def test_redshift_against_circular_orbit(orc, a):
    rin = orc.isco(a)
    for r in (rin * 1.01, 3.0 * rin, 17.0):
        E, L, Om, ut = circular_orbit(a, r)
        # L = 0 photon: g = 1 / u^t
        assert orc.redshift(a, r, 1.0, 0.0) == pytest.approx(1.0 / ut, rel=1e-13)
        for xi in (-6.0, -1.0, 2.5, 7.0):
            # stored momenta are the negated physical ones: p_t = E, p_phi = -L
            g = orc.redshift(a, r, 1.0, -xi)
            assert g == pytest.approx(1.0 / (ut * (1 - Om * xi)), rel=1e-13)
            assert orc.redshift(a, r, -1.0, xi) == g  # homogeneous of degree 0
    if a == 0.0:
        return
    assert orc.redshift(0.9, 10.0, 1.0, 0.0) == pytest.approx(0.8459362985, rel=1e-9)
