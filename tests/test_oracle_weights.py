"""Pins of per-edge weights in the oracle (Algorithm 2 gives every edge its
own rho_(a,b) and alpha_(a,b); here they are constant over each factor
group).

* the z-update is the rho-weighted mean of the incoming m, and with
  alpha = 1 the rho-weighted duals around every variable sum to zero at
  every iteration;
* the weights change the path, not the fixed point: unconstrained MPC with
  mixed rho and alpha still converges to the Riccati LQR solution, and a
  tiny SVM with mixed weights to the primal QP's minimiser;
* setting every group's weight to a value equals setting the graph's.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import pins


def _weighted(p, weights):
    """Copy of problem p with (rho, alpha) per group index."""
    groups = [dataclasses.replace(g, rho=weights.get(i, (None, None))[0],
                                  alpha=weights.get(i, (None, None))[1])
              for i, g in enumerate(p.groups)]
    return dataclasses.replace(p, groups=groups)


def _slot_rho(p):
    out = []
    for g in p.groups:
        r = p.rho if g.rho is None else g.rho
        out += [r] * int(p.var_dims[g.var_ids].sum())
    return np.asarray(out)


@pytest.mark.parametrize("case", ["packing", "svm"])
def test_weighted_mean_and_zero_dual_sums(case):
    if case == "packing":
        p = _weighted(W.packing(8, "square", 0.15, seed=31), {1: (2.0, None), 2: (3.0, None)})
    else:
        p = _weighted(W.svm(40, 3, seed=32), {0: (0.6, None), 1: (2.5, None)})
    g = O.OracleGraph(p)
    sz = g.slot_z
    w = _slot_rho(p)
    for _ in range(25):
        g.run(1)
        num = np.bincount(sz, weights=w * g.m, minlength=g.n_z)
        den = np.bincount(sz, weights=w, minlength=g.n_z)
        np.testing.assert_allclose(g.z, num / den, rtol=1e-13, atol=1e-14)
        du = np.bincount(sz, weights=w * g.u, minlength=g.n_z)
        # u = m - z cancels: its rounding scales with |z_b|
        scale = np.bincount(sz, weights=w * (np.abs(g.u) + np.abs(g.z[sz])), minlength=g.n_z) + 1e-30
        assert np.max(np.abs(du) / scale) < 1e-12


@pytest.mark.parametrize("seed", [1, 2])
def test_mixed_weights_keep_the_riccati_solution(seed):
    rng = np.random.default_rng(seed)
    T, n, m = 12, 4, 2
    A, B = W.mpc_system(rng, n, m)
    inst = W.MPCInstance(T, n, m, A, B, rng.standard_normal(n), np.ones(n), np.full(m, 0.1),
                         u_box=0.0)
    p = W.mpc_graph(inst, box=False)
    # groups: dynamics (first step, others), quadratic on x, quadratic on u
    p = _weighted(p, {0: (2.0, 1.0), 1: (2.0, 1.3), 2: (0.5, 0.8), 3: (1.5, 1.0)})
    g = O.OracleGraph(p)
    assert g.run(200000, tol=1e-12) > 0
    np.testing.assert_allclose(g.z, pins.riccati_lqr(inst), atol=1e-8)


def test_mixed_weights_keep_the_svm_optimum():
    p = _weighted(W.svm(8, 2, seed=33, sep=1.0), {0: (0.7, 1.2), 1: (2.0, None)})
    g = O.OracleGraph(p)
    g.run(400000, tol=1e-13)
    w_ref, _, _ = pins.svm_primal_slsqp(p.meta["a"], p.meta["y"], p.meta["C"])
    np.testing.assert_allclose(g.z[:2], w_ref, atol=1e-5)


def test_group_weights_equal_graph_weights():
    p = W.packing(6, "square", 0.2, seed=34)
    a = O.OracleGraph(p, rho=2.0, alpha=1.2)
    b = O.OracleGraph(_weighted(p, {i: (2.0, 1.2) for i in range(len(p.groups))}))
    a.run(30)
    b.run(30)
    assert np.array_equal(a.z, b.z) and np.array_equal(a.u, b.u)
    assert a.residuals() == b.residuals()
