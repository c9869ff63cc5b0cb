"""Pins for the oracle's proximal operators (paper eq. (3) and appendix).

Each operator is checked against its defining problem
argmin_s f(s) + rho/2 |s - n|^2 solved another way: scipy SLSQP on the
constrained form, a one-dimensional scan, or a KKT linear system.
"""
import numpy as np
import pytest

import oracle as O
from tests import pins


RHO = [0.5, 1.0, 3.0]


def _sq(x, n):
    return float(np.sum((np.asarray(x) - np.asarray(n)) ** 2))


@pytest.mark.parametrize("rho", RHO)
def test_nonoverlap_vs_constrained_minimum(rho):
    """App. A, first PO: projection onto |c1 - c2| >= r1 + r2.

    The output must be feasible (with equality when the input overlaps) and
    no point found by SLSQP from several starts may be closer.  The radius
    direction printed in the paper (+1) fails the feasibility check."""
    rng = np.random.default_rng(11)
    for _ in range(60):
        nv = np.concatenate([rng.random(2), rng.random(1) * 0.6,
                             rng.random(2), rng.random(1) * 0.6])
        x = O.prox("nonoverlap", [2, 1, 2, 1], [], rho, nv)
        gap = np.hypot(x[0] - x[3], x[1] - x[4]) - x[2] - x[5]
        L = np.hypot(nv[0] - nv[3], nv[1] - nv[4])
        if L >= nv[2] + nv[5]:
            np.testing.assert_array_equal(x, nv)
            continue
        assert abs(gap) < 1e-12
        best = np.inf
        con = dict(type="ineq",
                   fun=lambda s: np.hypot(s[0] - s[3], s[1] - s[4]) - s[2] - s[5])
        for start in (nv + 0.05 * rng.standard_normal(6), x, nv[[3, 4, 5, 0, 1, 2]]):
            s, _ = pins.slsqp(lambda s: _sq(s, nv), start, [con])
            if con["fun"](s) > -1e-9:
                best = min(best, _sq(s, nv))
        assert _sq(x, nv) <= best + 1e-9
        # feasible random perturbations never beat it
        for _ in range(50):
            s = x + 1e-3 * rng.standard_normal(6)
            if con["fun"](s) >= 0:
                assert _sq(s, nv) >= _sq(x, nv) - 1e-12


def test_nonoverlap_coincident_centres_convention():
    """When the two centres coincide the direction is taken as (1, 0)."""
    nv = np.array([0.3, 0.4, 0.1, 0.3, 0.4, 0.2])
    x = O.prox("nonoverlap", [2, 1, 2, 1], [], 1.0, nv)
    D = 0.3
    np.testing.assert_allclose(x, [0.3 - D / 4, 0.4, 0.1 - D / 4,
                                   0.3 + D / 4, 0.4, 0.2 - D / 4], atol=1e-15)


@pytest.mark.parametrize("rho", RHO)
def test_wall_is_halfspace_projection(rho):
    """App. A, second PO: projection onto Q^T (c - V) >= r (any |Q|)."""
    rng = np.random.default_rng(12)
    for _ in range(60):
        Q = rng.standard_normal(2) * rng.choice([1.0, 0.3, 2.0])
        V = rng.random(2)
        nv = rng.standard_normal(3)
        x = O.prox("wall", [2, 1], np.concatenate([Q, V]), rho, nv)
        con = dict(type="ineq", fun=lambda s: Q @ (s[:2] - V) - s[2])
        s, _ = pins.slsqp(lambda s: _sq(s, nv), nv.copy(), [con])
        np.testing.assert_allclose(x, s, atol=1e-7)
        # idempotent
        np.testing.assert_allclose(
            O.prox("wall", [2, 1], np.concatenate([Q, V]), rho, x), x, atol=1e-14)
    # unit normal, equal weights: the paper's printed closed form
    Q = np.array([0.6, 0.8]); V = np.array([0.2, 0.1]); nv = np.array([0.1, 0.1, 0.5])
    E = min(0.0, 0.5 * (Q @ (nv[:2] - V) - nv[2]))
    np.testing.assert_allclose(O.prox("wall", [2, 1], np.r_[Q, V], 1.0, nv),
                               nv + E * np.r_[-Q, 1.0], atol=1e-15)


@pytest.mark.parametrize("rho,gamma", [(1.0, 0.5), (3.0, 1.0), (0.7, 0.2)])
def test_radius_vs_scan(rho, gamma):
    """App. A, third PO with weight gamma and r >= 0: a fine scan of the
    1-D objective agrees with the closed form."""
    for nr in np.linspace(-0.5, 0.8, 27):
        x = O.prox("radius", [1], [gamma], rho, [nr])[0]
        grid = np.linspace(0.0, 5.0, 500001)
        obj = -0.5 * gamma * grid ** 2 + 0.5 * rho * (grid - nr) ** 2
        assert abs(x - grid[np.argmin(obj)]) < 2e-5
    with pytest.raises(ValueError):
        O.prox("radius", [1], [1.0], 1.0, [0.3])


@pytest.mark.parametrize("rho", RHO)
def test_quad_l2_box(rho):
    """App. B cost PO (1/2 sum q x^2), App. C norm-two PO, and the box."""
    rng = np.random.default_rng(13)
    nv = rng.standard_normal(5)
    q = rng.random(5) * 3
    x = O.prox("quad", [5], q, rho, nv)
    grad = q * x + rho * (x - nv)
    np.testing.assert_allclose(grad, 0.0, atol=1e-14)
    x = O.prox("l2", [1] * 5, [2.5], rho, nv)
    np.testing.assert_allclose(2.5 * x + rho * (x - nv), 0.0, atol=1e-14)
    x = O.prox("box", [5], [-0.3, 0.4], rho, nv)
    np.testing.assert_array_equal(x, np.clip(nv, -0.3, 0.4))


@pytest.mark.parametrize("rho", RHO)
def test_hinge_vs_slack_qp(rho):
    """Hinge factor C max(0, 1 - y(w.a + b)): equals the slack form
    min C xi + rho/2 |v - n|^2, xi >= 0, xi >= 1 - y(w.a + b)."""
    rng = np.random.default_rng(14)
    d = 4
    for _ in range(40):
        a = rng.standard_normal(d)
        y = rng.choice([-1.0, 1.0])
        C = rng.choice([0.3, 1.0, 4.0])
        nv = rng.standard_normal(d + 1) * 0.7
        x = O.prox("hinge", [1] * (d + 1), np.r_[a, y, C], rho, nv)

        def obj(v):
            return C * v[-1] + 0.5 * rho * _sq(v[:-1], nv)
        cons = [dict(type="ineq", fun=lambda v: v[-1]),
                dict(type="ineq", fun=lambda v: v[-1] - 1.0 + y * (v[:d] @ a + v[d]))]
        v0 = np.r_[nv, 1.0 + abs(nv).sum() * 3]
        s, _ = pins.slsqp(obj, v0, cons)
        np.testing.assert_allclose(x, s[:-1], atol=2e-6)


@pytest.mark.parametrize("rho", RHO)
def test_minerr_vs_scan(rho):
    """App. C minimal-error PO: argmin lambda xi + rho/2 (xi - n)^2, xi >= 0,
    per component, against a fine scan of the one-dimensional objective."""
    rng = np.random.default_rng(15)
    lam = 0.7
    nv = rng.standard_normal(7)
    x = O.prox("minerr", [7], [lam], rho, nv)
    grid = np.linspace(0.0, 4.0, 400001)
    for xi, ni in zip(x, nv):
        f = lam * grid + 0.5 * rho * (grid - ni) ** 2
        assert abs(xi - grid[np.argmin(f)]) < 2e-5
    with pytest.raises(Exception):
        O.prox("minerr", [1], [-1.0], rho, [0.3])


@pytest.mark.parametrize("rho", RHO)
def test_equal_vs_least_squares(rho):
    """App. C equality PO: min |w1 - n1|^2 + |w2 - n2|^2 over w1 = w2, solved
    as an overdetermined least-squares problem in the shared vector."""
    rng = np.random.default_rng(16)
    d = 5
    nv = rng.standard_normal(2 * d)
    x = O.prox("equal", [d, d], [], rho, nv)
    t, *_ = np.linalg.lstsq(np.vstack([np.eye(d), np.eye(d)]), nv, rcond=None)
    np.testing.assert_allclose(x, np.r_[t, t], atol=1e-14)


@pytest.mark.parametrize("rho", RHO)
def test_margin_vs_constrained_minimum(rho):
    """App. C one-point margin PO: the projection of (w, b, xi) onto
    y(w.x + b) >= 1 - xi.  Feasible inputs are returned unchanged, the
    output is feasible (active when the input was not) and SLSQP finds no
    closer feasible point."""
    rng = np.random.default_rng(17)
    d = 4
    active = 0
    for _ in range(40):
        xv = rng.standard_normal(d)
        y = rng.choice([-1.0, 1.0])
        nv = rng.standard_normal(d + 2) * 0.8
        out = O.prox("margin", [d, 1, 1], np.r_[xv, y], rho, nv)

        def g(v):
            return y * (v[:d] @ xv + v[d]) + v[d + 1] - 1.0
        if g(nv) >= 0:
            np.testing.assert_array_equal(out, nv)
            continue
        active += 1
        assert abs(g(out)) < 1e-12
        s, _ = pins.slsqp(lambda v: _sq(v, nv), nv.copy(), [dict(type="ineq", fun=g)])
        np.testing.assert_allclose(out, s, atol=2e-6)
    assert active > 5
    with pytest.raises(Exception):
        O.prox("margin", [d, 1, 1], np.r_[np.ones(d), 0.5], 1.0, np.zeros(d + 2))


def _lindyn_kkt(nv, n, m, A, B):
    """min |(x,u,x') - nv|^2 s.t. x' - A x - B u = 0 as one KKT system."""
    k = 2 * n + m
    Cm = np.hstack([-A, -B, np.eye(n)])
    K = np.block([[np.eye(k), Cm.T], [Cm, np.zeros((n, n))]])
    return np.linalg.solve(K, np.r_[nv, np.zeros(n)])[:k]


@pytest.mark.parametrize("n,m", [(4, 2), (8, 3), (12, 4), (1, 1)])
def test_lindyn_vs_kkt(n, m):
    """App. B dynamics PO: the projection onto x' = A x + B u."""
    rng = np.random.default_rng(15 + n)
    for _ in range(10):
        A = rng.standard_normal((n, n)); B = rng.standard_normal((n, m))
        nv = rng.standard_normal(2 * n + m)
        x = O.prox("lindyn", [n, m, n], np.r_[A.ravel(), B.ravel()], 1.0, nv)
        np.testing.assert_allclose(x, _lindyn_kkt(nv, n, m, A, B), atol=1e-11)
        np.testing.assert_allclose(x[n + m:], A @ x[:n] + B @ x[n:n + m], atol=1e-11)


@pytest.mark.parametrize("n,m", [(4, 2), (8, 3)])
def test_lindyn0_vs_kkt(n, m):
    """First step, x0 a parameter: projection of (u0, x1) onto x1 = A x0 + B u0."""
    rng = np.random.default_rng(25 + n)
    for _ in range(10):
        A = rng.standard_normal((n, n)); B = rng.standard_normal((n, m))
        x0 = rng.standard_normal(n)
        nv = rng.standard_normal(n + m)
        x = O.prox("lindyn0", [m, n], np.r_[A.ravel(), B.ravel(), x0], 1.0, nv)
        Cm = np.hstack([-B, np.eye(n)])
        K = np.block([[np.eye(n + m), Cm.T], [Cm, np.zeros((n, n))]])
        ref = np.linalg.solve(K, np.r_[nv, A @ x0])[:n + m]
        np.testing.assert_allclose(x, ref, atol=1e-11)
