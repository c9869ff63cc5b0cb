"""Integration pins for the oracle's Algorithm 2 (paper Sec. II).

* packing: one disk converges to the incircle (closed form); small packings
  end feasible; the graph has the paper's edge/factor/node counts;
* the z-update is the average of incoming m and, with u^0 = 0, the duals
  around every variable sum to zero at every iteration (follows from the
  z- and u-updates of Algorithm 2);
* MPC without the box equals the Riccati LQR solution; with the box it
  satisfies the active-set KKT conditions;
* tiny SVMs satisfy the KKT conditions with the duals recovered from u and
  match scipy's solution of the primal QP;
* the Fig. 1 example keeps the paper's edge order.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from tests import pins


def test_single_disk_incircle_triangle_and_square():
    p = W.packing(1, "triangle", 0.1, seed=3)
    g = O.OracleGraph(p)
    g.run(3000)
    np.testing.assert_allclose(g.z, [0.5, np.sqrt(3) / 6, np.sqrt(3) / 6], atol=1e-12)
    p = W.packing(1, "square", 0.1, seed=4)
    g = O.OracleGraph(p)
    g.run(3000)
    np.testing.assert_allclose(g.z, [0.5, 0.5, 0.5], atol=1e-12)


@pytest.mark.parametrize("N,S,shape", [(10, 3, "triangle"), (7, 4, "square"),
                                      (2000, 4, "square")])
def test_packing_graph_counts(N, S, shape):
    p = W.packing(N, shape, 0.02, seed=1)
    c = W.packing_counts(N, S)
    assert p.n_edges == c["edges"]
    assert p.n_factors == c["factors"]
    assert p.n_vars == c["var_nodes"]


def _check_invariants(problem, iters, alpha=None):
    g = O.OracleGraph(problem, alpha=alpha)
    sz = g.slot_z
    deg = np.bincount(sz, minlength=g.n_z).astype(float)
    for _ in range(iters):
        g.run(1)
        m, u, z = g.m, g.u, g.z
        zsum = np.bincount(sz, weights=m, minlength=g.n_z)
        np.testing.assert_allclose(z[deg > 0], (zsum / np.maximum(deg, 1))[deg > 0],
                                   rtol=1e-12, atol=1e-14)
        usum = np.bincount(sz, weights=u, minlength=g.n_z)
        assert np.max(np.abs(usum)) < 1e-12
        np.testing.assert_allclose(m, g.x + (u - (1.0 if alpha is None else alpha)
                                             * (g.x - z[sz])), atol=1e-13)


@pytest.mark.parametrize("alpha", [None, 1.5, 0.7])
def test_z_is_mean_of_m_and_duals_sum_to_zero(alpha):
    _check_invariants(W.packing(6, "triangle", 0.1, seed=21), 40, alpha)
    _check_invariants(W.svm(12, 3, seed=22), 20, alpha)


def test_small_packing_converges_feasible():
    p = W.workload("packing_tri10")
    g = O.OracleGraph(p)
    g.run(20000)
    obj = O.packing_objective(p, g.z)
    assert obj["max_violation"] < 1e-6
    r, s = g.residuals()
    assert r < 1e-6 and s < 1e-6
    # covers a substantial part of the triangle (area sqrt(3)/4)
    assert obj["area"] / (np.sqrt(3) / 4) > 0.7


@pytest.mark.parametrize("T,n,m,seed", [(12, 4, 2, 1), (25, 6, 3, 2), (8, 12, 4, 3)])
def test_unconstrained_mpc_equals_riccati(T, n, m, seed):
    rng = np.random.default_rng(seed)
    A, B = W.mpc_system(rng, n, m)
    inst = W.MPCInstance(T, n, m, A, B, rng.standard_normal(n),
                         np.ones(n), np.full(m, 0.1), u_box=0.0)
    g = O.OracleGraph(W.mpc_graph(inst, box=False))
    g.run(20000, tol=1e-12)
    np.testing.assert_allclose(g.z, pins.riccati_lqr(inst), atol=1e-8)


@pytest.mark.parametrize("seed", [5, 6, 7])
def test_boxed_mpc_satisfies_active_set_kkt(seed):
    rng = np.random.default_rng(seed)
    n, m, T = 4, 2, 15
    A, B = W.mpc_system(rng, n, m)
    inst = W.MPCInstance(T, n, m, A, B, 3.0 * rng.standard_normal(n),
                         np.ones(n), np.full(m, 0.1), u_box=0.5)
    g = O.OracleGraph(W.mpc_graph(inst))
    g.run(50000, tol=1e-12)
    z = g.z
    y, sign_bad, margin = pins.mpc_active_set_kkt(inst, z)
    assert np.max(np.abs(np.abs(z[[t * (n + m) + j for t in range(T) for j in range(m)]]))) > 0.5 - 1e-9
    np.testing.assert_allclose(z, y, atol=1e-8)
    assert sign_bad < 1e-8
    assert margin > -1e-9
    o = O.mpc_objective(inst, z)
    assert o["dyn_violation"] < 1e-8 and o["box_violation"] < 1e-10


@pytest.mark.parametrize("N,d,seed", [(8, 2, 31), (6, 3, 32), (10, 2, 33)])
def test_tiny_svm_kkt_and_qp(N, d, seed):
    p = W.svm(N, d, seed=seed, sep=1.0)
    g = O.OracleGraph(p)
    g.run(200000, tol=1e-13)
    z = g.z
    w, b = z[:d], z[d]
    a, y, C = p.meta["a"], p.meta["y"], p.meta["C"]
    # duals from the hinge factors' b-edge: beta_i = rho y_i u_(i,b)
    u = g.u.reshape(-1)[: N * (d + 1)].reshape(N, d + 1)
    beta = p.rho * y * u[:, d]
    assert np.all(beta > -1e-8) and np.all(beta < C + 1e-8)
    np.testing.assert_allclose(w, (beta * y) @ a, atol=1e-7)
    assert abs(np.sum(beta * y)) < 1e-7
    margin = y * (a @ w + b)
    for bi, mi in zip(beta, margin):
        if bi < 1e-6:
            assert mi > 1 - 1e-6
        elif bi > C - 1e-6:
            assert mi < 1 + 1e-6
        else:
            assert abs(mi - 1) < 1e-6
    w_ref, b_ref, f_ref = pins.svm_primal_slsqp(a, y, C)
    assert O.svm_objective(p, z) <= f_ref + 1e-7
    np.testing.assert_allclose(w, w_ref, atol=1e-5)


@pytest.mark.parametrize("N,d,seed", [(6, 2, 81), (8, 3, 82), (5, 2, 83)])
def test_copies_svm_graph_reaches_the_hinge_optimum(N, d, seed):
    """The paper's SVM graph (a copy of w per point tied by equality factors,
    margin, minimal-error and 1/N-weighted norm factors) solves the same
    problem as the hinge graph: at convergence every copy equals the
    hinge graph's w, b agrees, the slacks are the hinge losses, and w is the
    primal QP's minimiser."""
    p = W.svm_copies(N, d, seed=seed, sep=1.0)
    g = O.OracleGraph(p)
    g.run(400000, tol=1e-13)
    z = g.z
    Wc = z[:N * d].reshape(N, d)
    b, xi = z[N * d], z[N * d + 1:]
    h = O.OracleGraph(W.svm(N, d, seed=seed, sep=1.0))
    h.run(400000, tol=1e-13)
    for i in range(N):
        np.testing.assert_allclose(Wc[i], h.z[:d], atol=1e-7)
    assert abs(b - h.z[d]) < 1e-7
    a, y = p.meta["a"], p.meta["y"]
    np.testing.assert_allclose(xi, np.maximum(0.0, 1.0 - y * (a @ Wc[0] + b)), atol=1e-7)
    w_ref, _, _ = pins.svm_primal_slsqp(a, y, p.meta["C"])
    np.testing.assert_allclose(Wc[0], w_ref, atol=1e-5)


def test_copies_svm_graph_counts():
    N, d = 7, 3
    p = W.svm_copies(N, d, seed=84)
    assert p.n_vars == 2 * N + 1
    assert p.n_factors == 3 * N + (N - 1)
    assert p.n_edges == 3 * N + N + N + 2 * (N - 1)
    assert p.n_slots == N * (d + 2) + N + N * d + 2 * d * (N - 1)


def test_fig1_edge_order():
    """Edge arrays follow edge creation: for f1(w1,w2,w3) + f2(w1,w4,w5) +
    f3(w2,w5) + f4(w5) the order is (1,1),(1,2),(1,3),(2,1),(2,4),(2,5),
    (3,2),(3,5),(4,5); z has one entry per variable (five)."""
    facs = W.fig1_topology()
    groups = [W.FactorGroup("l2", np.array([f], np.int32), np.array([1.0]), True)
              for f in facs]
    p = W.Problem("fig1", np.ones(5, np.int32), groups, np.arange(5.0))
    g = O.OracleGraph(p)
    np.testing.assert_array_equal(g.slot_z, [0, 1, 2, 0, 3, 4, 1, 4, 4])
    assert g.n_z == 5


@pytest.mark.parametrize("seed", [51, 52, 53])
def test_dual_completion_is_the_converged_dual(seed):
    """At the solution z*, the completed duals equal the duals ADMM itself
    converges to, sum to zero around every variable, and make (z*, u0) a
    fixed point: the next iteration already meets the 1e-4 stopping rule."""
    from oracle import warmstart as WS
    inst = W.mpc_batch(1, seed=seed, T_range=(15, 30))[0]
    p = W.mpc_graph(inst)
    g = O.OracleGraph(p)
    g.run(200000, tol=1e-13)
    zs, us = g.z, g.u
    u0 = WS.dual_completion(inst, zs)
    assert u0.shape == us.shape
    np.testing.assert_allclose(u0, us, atol=1e-9)
    sz = g.slot_z
    np.testing.assert_allclose(np.bincount(sz, weights=u0, minlength=g.n_z), 0.0, atol=1e-12)
    h = O.OracleGraph(p)
    h.set_state(zs, u0)
    assert h.run(10000, tol=1e-4) == 1
    # completed duals of an arbitrary trajectory still sum to zero per variable
    zr = np.random.default_rng(seed).standard_normal(zs.shape)
    np.testing.assert_allclose(np.bincount(sz, weights=WS.dual_completion(inst, zr),
                                           minlength=g.n_z), 0.0, atol=1e-10)


def test_mlp_oracle_gradient_matches_finite_differences():
    from oracle import warmstart as WS
    rng = np.random.default_rng(3)
    shapes = [(5, 4), (5,), (6, 5), (6,), (3, 6), (3,)]
    params = [rng.standard_normal(s) * 0.5 for s in shapes]
    x = rng.standard_normal((7, 4))
    t = rng.standard_normal((7, 3))
    loss, grads = WS.mlp_loss_grad(params, x, t)
    h = 1e-6
    for p, gp in zip(params, grads):
        for idx in list(np.ndindex(p.shape))[:6]:
            old = p[idx]
            p[idx] = old + h
            lp, _ = WS.mlp_loss_grad(params, x, t)
            p[idx] = old - h
            lm, _ = WS.mlp_loss_grad(params, x, t)
            p[idx] = old
            assert abs((lp - lm) / (2 * h) - gp[idx]) < 1e-6


def test_bf16_rounding_matches_torch():
    """The oracle's bf16 rounding equals torch's float32 -> bfloat16 cast."""
    import torch
    from oracle import warmstart as WS
    rng = np.random.default_rng(9)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-20, 20, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 3.0e38]]).astype(np.float32)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(WS.bf16_round(x), ref)
