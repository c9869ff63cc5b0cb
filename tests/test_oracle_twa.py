"""Pins of the oracle's three-weight variant (Sec. II: per-edge weights with
improved update schemes; every message weight is 0 or rho here, see the
oracle's header).  CPU only."""
import numpy as np
import pytest
from scipy.optimize import minimize

import oracle as O
import workloads as W
from tests.helpers import slot_z


def _pair_problem(z0):
    """Two disks in the unit square (pair, four walls each, radius weight
    gamma = 0.5) from a given start."""
    p = W.packing(2, "square", 0.01, seed=1)
    p.z0 = np.asarray(z0, dtype=np.float64)
    return p


@pytest.mark.parametrize("make", [lambda: W.svm(400, 5, seed=3),
                                  lambda: W.mpc_graph(W.mpc_batch(1, seed=41)[0]),
                                  lambda: W.svm_copies(60, 4, seed=5)])
def test_without_constraint_factors_it_is_algorithm2(make):
    """No hinge, margin, dynamics or norm factor ever sends weight 0: the
    three-weight run is Algorithm 2 bit for bit."""
    p = make()
    a, b = O.OracleGraph(p), O.OracleGraph(p, twa=True)
    a.run(60)
    b.run(60)
    assert np.array_equal(a.z, b.z) and np.array_equal(a.u, b.u) and np.array_equal(a.x, b.x)
    assert np.all(b.wr == 1.0)


def test_first_iterations_by_hand():
    """Two small disks far apart and far from the walls: every pair and wall
    constraint is inactive, so only the radius factors send weight.  The
    centres keep their values (no factor has an opinion), each radius
    follows its radius factor alone, r <- rho r / (rho - gamma) = 2 r, and
    every u stays 0.  Plain ADMM averages the radius over its six edges
    instead: (2 + 5) r / 6."""
    z0 = [0.3, 0.3, 0.01, 0.7, 0.7, 0.01]
    p = _pair_problem(z0)
    o = O.OracleGraph(p, twa=True)
    for k in (1, 2, 3):
        o.run(1)
        r = 0.01 * 2.0 ** k
        np.testing.assert_array_equal(o.z, [0.3, 0.3, r, 0.7, 0.7, r])
        assert np.all(o.u == 0.0)
    wr = o.wr
    # slots: pair (6), then walls (4 per disk x 3 slots), then radii (1 each)
    assert np.all(wr[:6 + 24] == 0.0) and np.all(wr[30:] == 1.0)
    q = O.OracleGraph(p)
    q.run(1)
    assert abs(q.z[2] - 7.0 / 6.0 * 0.01) < 1e-15


def test_free_nonoverlap_prox():
    """Zero received weight on c1 only: c1 alone absorbs the overlap D along
    the centre line and the pair ends in contact; both centres free: equal
    halves.  Against the weighted projection solved numerically with the
    free edges' weight 1e-6 (the limit as it goes to 0)."""
    rng = np.random.default_rng(0)
    for trial in range(200):
        nv = np.r_[rng.uniform(0, 1, 2), rng.uniform(0.1, 0.3), rng.uniform(0, 1, 2),
                   rng.uniform(0.1, 0.3)]
        for free in ([0], [2], [0, 2]):
            wl = np.ones(6)
            for e in free:
                wl[[0, 1] if e == 0 else [3, 4]] = 0.0
            out = O.prox_free("nonoverlap", None, wl, nv)
            c1, r1, c2, r2 = out[:2], out[2], out[3:5], out[5]
            L0 = np.hypot(*(nv[3:5] - nv[:2]))
            D = max(0.0, nv[2] + nv[5] - L0)
            assert r1 == nv[2] and r2 == nv[5]
            if D == 0.0:
                np.testing.assert_array_equal(out, nv)
                continue
            assert abs(np.hypot(*(c2 - c1)) - (r1 + r2)) < 1e-12
            if trial < 20:       # numerical projection, free weights 1e-6
                w = np.ones(6)
                w[wl == 0.0] = 1e-6
                res = minimize(lambda x: 0.5 * np.sum(w * (x - nv) ** 2), out, jac=lambda x: w * (x - nv),
                               constraints=[dict(type="ineq",
                                                 fun=lambda x: np.hypot(x[3] - x[0], x[4] - x[1]) - x[2] - x[5])],
                               method="SLSQP", options=dict(ftol=1e-16, maxiter=500))
                assert np.max(np.abs(res.x - out)) < 1e-4 * max(D, 1e-3)


def test_free_wall_prox():
    rng = np.random.default_rng(1)
    Q = np.array([np.sqrt(3) / 2, -0.5])
    V = np.zeros(2)
    par = np.r_[Q, V]
    for _ in range(200):
        nv = np.r_[rng.uniform(-0.3, 0.3, 2), rng.uniform(0.05, 0.3)]
        g = Q @ (nv[:2] - V) - nv[2]
        out = O.prox_free("wall", par, np.array([0.0, 0.0, 1.0]), nv)
        if g >= 0:
            np.testing.assert_array_equal(out, nv)
            continue
        assert out[2] == nv[2]
        assert abs(Q @ (out[:2] - V) - out[2]) < 1e-14
        d = out[:2] - nv[:2]
        assert abs(d[0] * Q[1] - d[1] * Q[0]) < 1e-15          # moved along Q
        both = O.prox_free("wall", par, np.zeros(3), nv)
        np.testing.assert_allclose(both, O.prox("wall", [2, 1], par, 1.0, nv), rtol=0, atol=1e-15)


def _step_invariants(p, iters):
    o = O.OracleGraph(p, twa=True)
    sz = slot_z(p)
    for _ in range(iters):
        zp = o.z
        o.run(1)
        z, m, u, wr = o.z, o.m, o.u, o.wr
        assert set(np.unique(wr)) <= {0.0, 1.0}
        num = np.bincount(sz, weights=wr * m, minlength=p.n_scalars)
        den = np.bincount(sz, weights=wr, minlength=p.n_scalars)
        want = np.where(den > 0, num / np.where(den > 0, den, 1.0), zp)
        np.testing.assert_allclose(z, want, rtol=1e-13, atol=1e-15)
        assert np.all(u[wr == 0.0] == 0.0)


def test_zupdate_and_dual_reset_every_iteration():
    _step_invariants(W.packing(30, "square", 0.1, seed=7), 40)
    _step_invariants(W.workload("packing_tri10"), 40)


@pytest.mark.parametrize("N,shape,seed", [(1, "triangle", 0), (2, "square", 1), (3, "triangle", 2),
                                          (4, "triangle", 5), (6, "triangle", 6),
                                          (10, "triangle", 1000), (15, "triangle", 12)])
def test_ends_feasible_on_tiny_packings(N, shape, seed):
    """Run to a fixed point: no overlap, every disk inside the container, and
    one disk in the triangle ends as its incircle (r = sqrt(3)/6).  (Packing
    is nonconvex: on some small square instances neither Algorithm 2 nor
    this variant settles; these instances settle under both.)"""
    p = W.packing(N, shape, 0.1 if shape == "triangle" else 0.05, seed=seed)
    o = O.OracleGraph(p, twa=True)
    o.run(20000)
    f = O.packing_objective(p, o.z)
    assert f["max_violation"] < 1e-12, f
    r, s = o.residuals()
    assert r < 1e-12 and s < 1e-12
    if N == 1:
        assert abs(o.z[2] - np.sqrt(3) / 6) < 1e-9
        np.testing.assert_allclose(o.z[:2], [0.5, np.sqrt(3) / 6], atol=1e-9)
