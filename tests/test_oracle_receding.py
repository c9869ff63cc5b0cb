"""Pins of the oracle's receding-horizon cycle (paper Sec. V-B: each
controller cycle updates the current state and continues the ADMM from the
previous cycle's solution).

* (z, u) is the whole ADMM state when alpha = 1: stopping after k1
  iterations and continuing from (z, u) gives the k1 + k2 iterate;
* the shift keeps a dynamically feasible trajectory feasible from the new
  initial state (x0' = A x0 + B u_0 is then the old x_1), and a disturbance
  enters only x0';
* the shifted duals still sum to zero around every variable (the invariant
  that Algorithm 2 keeps from u^0 = 0);
* continuing from the shifted solution needs fewer iterations than a cold
  start of the next cycle's problem.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import warmstart as WS


def _inst(seed, T=(15, 40), box=1.0):
    inst = W.mpc_batch(1, seed=seed, T_range=T)[0]
    return dataclasses.replace(inst, u_box=box)


def _feasible_z(inst, x0, rng):
    """A trajectory that meets the dynamics exactly (random inputs)."""
    T, n, m = inst.T, inst.n, inst.m
    z = np.zeros((T, n + m))
    x = np.asarray(x0, np.float64)
    for t in range(T):
        u = rng.standard_normal(m)
        x = inst.A @ x + inst.B @ u
        z[t, :m], z[t, m:] = u, x
    return z


def _dyn_violation(inst, x0, z):
    T, n, m = inst.T, inst.n, inst.m
    z = z.reshape(T, n + m)
    x = np.asarray(x0, np.float64)
    worst = 0.0
    for t in range(T):
        worst = max(worst, np.max(np.abs(z[t, m:] - inst.A @ x - inst.B @ z[t, :m])))
        x = z[t, m:]
    return worst


@pytest.mark.parametrize("seed", [31, 32])
def test_state_is_z_and_u(seed):
    inst = _inst(seed)
    p = W.mpc_graph(inst)
    g = O.OracleGraph(p)
    g.run(60)
    h = O.OracleGraph(p)
    h.run(25)
    k = O.OracleGraph(p)
    k.set_state(h.z, h.u)
    k.run(35)
    np.testing.assert_allclose(k.z, g.z, rtol=0, atol=1e-12)
    np.testing.assert_allclose(k.u, g.u, rtol=0, atol=1e-12)


@pytest.mark.parametrize("T", [1, 2, 17])
def test_shift_keeps_feasible_trajectory_feasible(T):
    rng = np.random.default_rng(40 + T)
    inst = _inst(41, T=(T, T))
    z = _feasible_z(inst, inst.x0, rng)
    assert _dyn_violation(inst, inst.x0, z) < 1e-12
    x0n, zn, _ = WS.receding_shift(inst, inst.x0, z.ravel())
    np.testing.assert_allclose(x0n, z[0, inst.m:], rtol=0, atol=1e-12)
    assert _dyn_violation(inst, x0n, zn) < 1e-12
    # the new last step has no input
    assert np.all(zn.reshape(T, -1)[T - 1, :inst.m] == 0.0)
    w = rng.standard_normal(inst.n)
    x0w, zw, _ = WS.receding_shift(inst, inst.x0, z.ravel(), w=w)
    np.testing.assert_allclose(x0w - x0n, w, rtol=0, atol=1e-12)
    np.testing.assert_array_equal(zw, zn)


@pytest.mark.parametrize("seed,box", [(33, 1.0), (34, 0.0)])
def test_shifted_duals_sum_to_zero(seed, box):
    inst = _inst(seed, box=box)
    p = W.mpc_graph(inst, box=box > 0)
    g = O.OracleGraph(p)
    g.run(80)
    sz = g.slot_z
    np.testing.assert_allclose(np.bincount(sz, weights=g.u, minlength=g.n_z), 0.0, atol=1e-12)
    _, _, un = WS.receding_shift(inst, inst.x0, g.z, g.u)
    assert un.shape == g.u.shape
    np.testing.assert_allclose(np.bincount(sz, weights=un, minlength=g.n_z), 0.0, atol=1e-12)
    # the moved blocks are copies: every value of the new duals is an old one or 0
    assert np.all(np.isin(un[un != 0.0], g.u))


@pytest.mark.parametrize("seed", [35, 36, 37])
def test_shifted_warm_start_beats_cold(seed):
    inst = _inst(seed, T=(30, 50))
    p = W.mpc_graph(inst)
    g = O.OracleGraph(p)
    assert g.run(20000, tol=1e-4) > 0
    x0n, zn, un = WS.receding_shift(inst, inst.x0, g.z, g.u)
    nxt = dataclasses.replace(inst, x0=x0n)
    q = W.mpc_graph(nxt)
    cold = O.OracleGraph(q).run(20000, tol=1e-4)
    h = O.OracleGraph(q)
    h.set_state(zn, un)
    warm = h.run(20000, tol=1e-4)
    assert 0 < warm < cold, (warm, cold)
