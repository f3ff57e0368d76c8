"""Pins of the oracle's metric, Hamiltonian and right-hand side (CPU only).

Each check ties the oracle to something other than its own formulas:
Ricci-flatness (Kerr is a vacuum solution), textbook special cases
(Schwarzschild, horizon, ergosphere, Lense-Thirring frame dragging, the
Kerr determinant identity), a numerical matrix inverse for Eq. (1), and
finite differences of H for Hamilton's equations, Eqs. (2)-(3).
"""
import math

import numpy as np
import pytest

POINTS = [(0.0, 6.0, 1.1), (0.5, 3.7, 0.4), (0.9, 2.9, 2.2), (0.998, 1.6, 1.3), (0.7, 40.0, 0.2)]


def full(g):
    G = np.zeros((4, 4))
    G[0, 0], G[0, 3], G[3, 0], G[1, 1], G[2, 2], G[3, 3] = g[0], g[1], g[1], g[2], g[3], g[4]
    return G


@pytest.mark.parametrize("a,r,th", POINTS)
def test_metric_derivatives_match_finite_differences(orc, a, r, th):
    m = orc.make_metric(a)
    g, gr, gt = orc.metric_eval(m, r, th)
    e = 1e-5
    fr = (orc.metric_eval(m, r + e, th)[0] - orc.metric_eval(m, r - e, th)[0]) / (2 * e)
    ft = (orc.metric_eval(m, r, th + e)[0] - orc.metric_eval(m, r, th - e)[0]) / (2 * e)
    scale = np.abs(g).max()
    assert np.allclose(gr, fr, rtol=1e-7, atol=1e-8 * scale)
    assert np.allclose(gt, ft, rtol=1e-7, atol=1e-8 * scale)
    # mixed second derivative of the smooth (tabulated) components
    c0 = orc.kerr_smooth_components(a, r, th)
    cp = orc.kerr_smooth_components(a, r, th + e)
    cm = orc.kerr_smooth_components(a, r, th - e)
    frt = (cp[:, 1] - cm[:, 1]) / (2 * e)
    assert np.allclose(c0[:, 3], frt, rtol=1e-6, atol=1e-8 * np.abs(c0[:, 0]).max())


def christoffel(orc, m, r, th):
    g, gr, gt = orc.metric_eval(m, r, th)
    G = full(g)
    Gi = np.linalg.inv(G)
    dG = np.zeros((4, 4, 4))  # dG[c] = d_c g
    dG[1] = full(gr)
    dG[2] = full(gt)
    Gam = np.zeros((4, 4, 4))
    for a_ in range(4):
        for b in range(4):
            for c in range(4):
                Gam[a_, b, c] = 0.5 * sum(Gi[a_, d] * (dG[b][d, c] + dG[c][d, b] - dG[d][b, c]) for d in range(4))
    return Gam


@pytest.mark.parametrize("a,r,th", POINTS[:4])
def test_kerr_is_ricci_flat(orc, a, r, th):
    """Kerr solves the vacuum field equations: R_bd = 0.  Any mistake in a
    component of the closed-form metric (a dropped term, a wrong sign) leaves
    curvature of order M / r^3."""
    m = orc.make_metric(a)
    e = 1e-3
    Gam = christoffel(orc, m, r, th)
    dGam = np.zeros((4, 4, 4, 4))  # dGam[c] = d_c Gamma, 4th-order central differences

    def d5(f):
        return (-f(2 * e) + 8 * f(e) - 8 * f(-e) + f(-2 * e)) / (12 * e)

    dGam[1] = d5(lambda h: christoffel(orc, m, r + h, th))
    dGam[2] = d5(lambda h: christoffel(orc, m, r, th + h))
    Ric = np.zeros((4, 4))
    for b in range(4):
        for d in range(4):
            s = 0.0
            for a_ in range(4):
                s += dGam[a_][a_, b, d] - dGam[d][a_, a_, b]
                for c in range(4):
                    s += Gam[a_, a_, c] * Gam[c, b, d] - Gam[a_, d, c] * Gam[c, a_, b]
            Ric[b, d] = s
    # compare in an orthonormal-like normalisation: R_bd / sqrt|g_bb g_dd| against
    # the curvature scale M / r^3 of the exterior
    g, _, _ = orc.metric_eval(m, r, th)
    diag = np.abs(np.diag(full(g)))
    Rn = Ric / np.sqrt(np.outer(diag, diag))
    curv = 1.0 / r ** 3
    assert np.abs(Rn).max() < 1e-6 * curv, Rn


def test_schwarzschild_special_case(orc):
    m = orc.make_metric(0.0)
    for r, th in [(3.0, 0.7), (10.0, 1.5), (250.0, 2.9)]:
        g, _, _ = orc.metric_eval(m, r, th)
        f = 1 - 2 / r
        assert np.allclose(g, [-f, 0.0, 1 / f, r * r, r * r * math.sin(th) ** 2], rtol=1e-15, atol=0)


@pytest.mark.parametrize("a", [0.3, 0.9, 0.998])
def test_kerr_landmarks(orc, a):
    m = orc.make_metric(a)
    # horizon: larger root of Delta = r^2 - 2r + a^2
    rp = max(np.roots([1.0, -2.0, a * a]).real)
    assert orc.horizon(a) == pytest.approx(rp, rel=1e-14)
    g, _, _ = orc.metric_eval(m, rp * (1 + 1e-9), 1.0)
    assert 1.0 / g[2] < 1e-7  # g^rr -> 0 at the horizon
    # ergosphere: g_tt = 0 at r = 1 + sqrt(1 - a^2 cos^2)
    for th in (0.3, 1.0, 1.5):
        rE = 1 + math.sqrt(1 - a * a * math.cos(th) ** 2)
        g, _, _ = orc.metric_eval(m, rE, th)
        assert abs(g[0]) < 1e-14
    # determinant identity: det g = -Sigma^2 sin^2(theta)
    for r, th in [(2.5, 0.8), (17.0, 2.0)]:
        g, _, _ = orc.metric_eval(m, r, th)
        S = r * r + a * a * math.cos(th) ** 2
        assert np.linalg.det(full(g)) == pytest.approx(-S * S * math.sin(th) ** 2, rel=1e-12)
    # Lense-Thirring frame dragging omega -> 2 a / r^3 far away
    r = 1e4
    g, _, _ = orc.metric_eval(m, r, 1.2)
    omega = -g[1] / g[4]
    assert omega * r ** 3 / (2 * a) == pytest.approx(1.0, rel=1e-3)


def random_momenta(rng):
    return rng.normal(size=4)


@pytest.mark.parametrize("a,r,th", POINTS)
def test_hamiltonian_is_half_inverse_metric_contraction(orc, a, r, th):
    """Eq. (1) against a numerical matrix inverse."""
    m = orc.make_metric(a)
    rng = np.random.default_rng(7)
    g, _, _ = orc.metric_eval(m, r, th)
    Gi = np.linalg.inv(full(g))
    for _ in range(4):
        p = random_momenta(rng)
        q = np.array([0.3, r, th, 1.1, *p])
        Href = 0.5 * p @ Gi @ p
        assert orc.hamiltonian(m, q) == pytest.approx(Href, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("a,r,th", POINTS)
def test_rhs_is_hamiltons_equations(orc, a, r, th):
    """Eqs. (2)-(3): the right-hand side equals (dH/dp, -dH/dx) of the oracle's
    own Eq. (1), differentiated numerically (4th-order central differences)."""
    m = orc.make_metric(a)
    rng = np.random.default_rng(11)
    for _ in range(3):
        q = np.array([0.3, r, th, 1.1, *random_momenta(rng)])
        d = orc.rhs(m, q)
        grad = np.zeros(8)
        for k in range(8):
            e = 1e-4 * max(1.0, abs(q[k]))
            def H(x):
                qq = q.copy(); qq[k] = x
                return orc.hamiltonian(m, qq)
            grad[k] = (-H(q[k] + 2 * e) + 8 * H(q[k] + e) - 8 * H(q[k] - e) + H(q[k] - 2 * e)) / (12 * e)
        expect = np.concatenate([grad[4:], -grad[:4]])
        scale = np.abs(expect).max()
        assert np.allclose(d, expect, rtol=1e-7, atol=1e-9 * scale), (d, expect)
        assert d[4] == 0.0 and d[7] == 0.0  # t and phi are cyclic: E and L conserved exactly
