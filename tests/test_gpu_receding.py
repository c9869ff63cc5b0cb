"""GPU parity of the receding-horizon pieces of the batched MPC solver
(paper Sec. V-B: each controller cycle updates the current state and
continues the ADMM from the previous cycle's solution).

* solve_state returns the per-edge duals u = m - z: they equal the oracle's
  after the same iterations, and continuing from (z, u) gives the iterate a
  single longer solve reaches;
* the shift kernel equals the oracle's ``receding_shift``: copies and zeros
  bit for bit, the two matrix-vector products (x0' and the new last state)
  to FP32 rounding;
* a closed loop of solve + shift cycles follows the oracle's closed loop;
* continuing from the shifted solution needs fewer iterations than a cold
  start of each cycle.
"""
import dataclasses

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import warmstart as WS
from tests.helpers import rel
from tests.test_gpu_mpc import _edge_instances, _gpu_u_to_oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mpc():
    from paper_1603_02526_amd import mpc as M
    return M


def _dev(a, dtype=torch.float32):
    return torch.tensor(np.asarray(a), dtype=dtype, device="cuda")


def _zeros(n, dtype=torch.float32):
    return torch.zeros(int(n), dtype=dtype, device="cuda")


def _zsize(i):
    return i.T * (i.n + i.m)


def _usize(i):
    return 3 * i.T * (i.n + i.m)


def test_solve_state_duals_and_continuation():
    M = _mpc()
    insts = _edge_instances() + W.mpc_batch(12, seed=71)
    b = M.MPCBatch(insts)
    x0 = _dev(b.pack_x0([i.x0 for i in insts]))
    z1, u1, it = _zeros(b.z_total), _zeros(b.u_total), _zeros(b.n_inst, torch.int32)
    b.solve_state(x0, z1, it, u_out=u1, tol=1e-30, max_iter=30)
    z2, u2 = _zeros(b.z_total), _zeros(b.u_total)
    b.solve_state(x0, z2, it, z_init=z1, u_init=u1, u_out=u2, tol=1e-30, max_iter=20)
    z50 = _zeros(b.z_total)
    b.solve_state(x0, z50, it, tol=1e-30, max_iter=50)
    # the plain solve entry point gives the same z as solve_state
    z50b = _zeros(b.z_total)
    b.solve(x0, z50b, it, tol=1e-30, max_iter=50)
    torch.cuda.synchronize()
    assert torch.equal(z50, z50b)
    z1h, u1h = z1.cpu().numpy(), u1.cpu().numpy()
    z2h, z50h = z2.cpu().numpy(), z50.cpu().numpy()
    for i, inst in enumerate(insts):
        g = O.OracleGraph(W.mpc_graph(inst, box=inst.u_box > 0))
        g.run(30)
        zg = z1h[b.z_off[i]:b.z_off[i] + _zsize(inst)]
        ug = _gpu_u_to_oracle(inst, u1h[b.u_off[i]:b.u_off[i] + _usize(inst)].astype(np.float64))
        assert rel(zg, g.z) < 1e-4, (i, rel(zg, g.z))
        assert rel(ug, g.u) < 1e-4, (i, rel(ug, g.u))
        g.run(20)
        zc = z2h[b.z_off[i]:b.z_off[i] + _zsize(inst)]
        zs = z50h[b.z_off[i]:b.z_off[i] + _zsize(inst)]
        assert rel(zc, zs) < 1e-5, (i, rel(zc, zs))
        assert rel(zc, g.z) < 1e-4, (i, rel(zc, g.z))


def test_shift_matches_oracle():
    M = _mpc()
    insts = _edge_instances() + W.mpc_batch(10, seed=72)
    b = M.MPCBatch(insts)
    rng = np.random.default_rng(73)
    x0 = rng.standard_normal(b.x0_total).astype(np.float32)
    z = rng.standard_normal(b.z_total).astype(np.float32)
    u = rng.standard_normal(b.u_total).astype(np.float32)
    w = (0.1 * rng.standard_normal(b.x0_total)).astype(np.float32)
    x0n, zn, un = _zeros(b.x0_total), _zeros(b.z_total), _zeros(b.u_total)
    b.shift(_dev(x0), _dev(z), x0n, z_next=zn, u=_dev(u), u_next=un, w=_dev(w))
    # z alone, no disturbance
    x0n2, zn2 = _zeros(b.x0_total), _zeros(b.z_total)
    b.shift(_dev(x0), _dev(z), x0n2, z_next=zn2)
    torch.cuda.synchronize()
    x0n, zn, un = x0n.cpu().numpy(), zn.cpu().numpy(), un.cpu().numpy()
    x0n2, zn2 = x0n2.cpu().numpy(), zn2.cpu().numpy()
    assert np.array_equal(zn, zn2)
    for i, inst in enumerate(insts):
        T, n, m = inst.T, inst.n, inst.m
        k = n + m
        xo = slice(b.x0_off[i], b.x0_off[i] + n)
        zi = z[b.z_off[i]:b.z_off[i] + _zsize(inst)].astype(np.float64)
        ug = u[b.u_off[i]:b.u_off[i] + _usize(inst)].astype(np.float64)
        uo = _gpu_u_to_oracle(inst, ug)
        ex0, ez, eu = WS.receding_shift(inst, x0[xo].astype(np.float64), zi, uo, w=w[xo])
        ex0b, _, _ = WS.receding_shift(inst, x0[xo].astype(np.float64), zi)
        assert rel(x0n[xo], ex0) < 1e-6, (i, rel(x0n[xo], ex0))
        assert rel(x0n2[xo], ex0b) < 1e-6, (i, rel(x0n2[xo], ex0b))
        zg = zn[b.z_off[i]:b.z_off[i] + _zsize(inst)].astype(np.float64)
        # steps moved forward are copies; the new last step: u = 0, x = A x_T
        np.testing.assert_array_equal(zg[:(T - 1) * k], ez[:(T - 1) * k])
        np.testing.assert_array_equal(zg[(T - 1) * k:(T - 1) * k + m], 0.0)
        assert rel(zg[(T - 1) * k + m:], ez[(T - 1) * k + m:]) < 1e-6
        un_i = un[b.u_off[i]:b.u_off[i] + _usize(inst)].astype(np.float64)
        np.testing.assert_array_equal(_gpu_u_to_oracle(inst, un_i), eu)
        # step 0 has no x_t edge: its slots are cleared
        np.testing.assert_array_equal(un_i.reshape(T, 3 * k)[0, :n], 0.0)


def test_closed_loop_follows_oracle():
    """Three controller cycles of 40 iterations each (fixed counts, so both
    sides run the same iterations), with a disturbance on the plant."""
    M = _mpc()
    insts = _edge_instances()[:8] + W.mpc_batch(8, seed=74)
    b = M.MPCBatch(insts)
    rng = np.random.default_rng(75)
    ws = [(0.05 * rng.standard_normal(b.x0_total)).astype(np.float32) for _ in range(3)]
    x0 = _dev(b.pack_x0([i.x0 for i in insts]))
    z, u = None, None
    it = _zeros(b.n_inst, torch.int32)
    gpu_z = []
    for c in range(3):
        zo, uo = _zeros(b.z_total), _zeros(b.u_total)
        b.solve_state(x0, zo, it, z_init=z, u_init=u, u_out=uo, tol=1e-30, max_iter=40)
        gpu_z.append(zo.cpu().numpy())
        x0n, zn, un = _zeros(b.x0_total), _zeros(b.z_total), _zeros(b.u_total)
        b.shift(x0, zo, x0n, z_next=zn, u=uo, u_next=un, w=_dev(ws[c]))
        x0, z, u = x0n, zn, un
    torch.cuda.synchronize()
    for i, inst in enumerate(insts):
        xo = slice(b.x0_off[i], b.x0_off[i] + inst.n)
        cur = inst
        zs = us = None
        for c in range(3):
            g = O.OracleGraph(W.mpc_graph(cur, box=cur.u_box > 0))
            if zs is not None:
                g.set_state(zs, us)
            g.run(40)
            zg = gpu_z[c][b.z_off[i]:b.z_off[i] + _zsize(inst)]
            assert rel(zg, g.z) < 1e-4, (i, c, rel(zg, g.z))
            x0n, zs, us = WS.receding_shift(cur, cur.x0, g.z, g.u, w=ws[c][xo])
            cur = dataclasses.replace(cur, x0=x0n)


def test_shifted_warm_start_beats_cold_on_gpu():
    M = _mpc()
    insts = W.mpc_batch(64, seed=76)
    b = M.MPCBatch(insts)
    rng = np.random.default_rng(77)
    x0 = _dev(b.pack_x0([i.x0 for i in insts]))
    z, u, it = _zeros(b.z_total), _zeros(b.u_total), _zeros(b.n_inst, torch.int32)
    b.solve_state(x0, z, it, u_out=u, tol=1e-4, max_iter=10000)
    w = _dev((0.1 * rng.standard_normal(b.x0_total)).astype(np.float32))
    x0n, zn, un = _zeros(b.x0_total), _zeros(b.z_total), _zeros(b.u_total)
    b.shift(x0, z, x0n, z_next=zn, u=u, u_next=un, w=w)
    zc, itc = _zeros(b.z_total), _zeros(b.n_inst, torch.int32)
    b.solve_state(x0n, zc, itc, tol=1e-4, max_iter=10000)
    zw, itw = _zeros(b.z_total), _zeros(b.n_inst, torch.int32)
    b.solve_state(x0n, zw, itw, z_init=zn, u_init=un, tol=1e-4, max_iter=10000)
    torch.cuda.synchronize()
    itc, itw = itc.cpu().numpy(), itw.cpu().numpy()
    assert np.all(itc > 0) and np.all(itw > 0)
    assert itw.mean() < 0.9 * itc.mean(), (itw.mean(), itc.mean())
    # both reach the same solution (strictly convex problem)
    assert rel(zw.cpu().numpy(), zc.cpu().numpy()) < 1e-2


def test_argument_errors():
    M = _mpc()
    from paper_1603_02526_amd.admm import AdmmError
    insts = W.mpc_batch(3, seed=78)
    b = M.MPCBatch(insts)
    x0 = _dev(b.pack_x0([i.x0 for i in insts]))
    z, u, it = _zeros(b.z_total), _zeros(b.u_total), _zeros(b.n_inst, torch.int32)
    with pytest.raises(AdmmError):
        b.solve_state(x0, z, it, u_init=u, tol=1e-4)       # u_init without z_init
    with pytest.raises(AdmmError):
        b.solve_state(x0, z, it, z_init=z, tol=1e-4)       # z_out is z_init
    with pytest.raises(AdmmError):
        b.shift(x0, z, x0)                                   # x0_next is x0
    with pytest.raises(AdmmError):
        b.shift(x0, z, _zeros(b.x0_total), u=u)              # u without u_next


def test_full_batch_cycle_from_common_state():
    """One controller cycle of the benchmark's 4096-instance batch, checked
    on sampled instances from a common state: the oracle takes the GPU's
    cycle-0 solution and duals, applies its own shift with the same
    disturbance and solves to the same tolerance."""
    M = _mpc()
    insts = W.mpc_batch(4096, seed=1003)
    b = M.MPCBatch(insts)
    x0 = _dev(b.pack_x0([i.x0 for i in insts]))
    z, u, it = _zeros(b.z_total), _zeros(b.u_total), _zeros(b.n_inst, torch.int32)
    b.solve_state(x0, z, it, u_out=u, tol=1e-4, max_iter=10000)
    w = W.mpc_disturbance(b.x0_total, 1, seed=1103, sd=0.1)[0]
    x0n, zn, un = _zeros(b.x0_total), _zeros(b.z_total), _zeros(b.u_total)
    b.shift(x0, z, x0n, z_next=zn, u=u, u_next=un, w=_dev(w))
    zw, itw = _zeros(b.z_total), _zeros(b.n_inst, torch.int32)
    b.solve_state(x0n, zw, itw, z_init=zn, u_init=un, tol=1e-4, max_iter=10000)
    torch.cuda.synchronize()
    itw = itw.cpu().numpy()
    assert np.all(itw > 0)
    zh, uh, zwh = z.cpu().numpy(), u.cpu().numpy(), zw.cpu().numpy()
    rng = np.random.default_rng(6)
    sample = list(np.argsort(-itw)[:3]) + list(rng.choice(4096, 10, replace=False))
    for i in sorted(set(int(s) for s in sample)):
        inst = insts[i]
        xo = slice(b.x0_off[i], b.x0_off[i] + inst.n)
        zi = zh[b.z_off[i]:b.z_off[i] + _zsize(inst)].astype(np.float64)
        ui = _gpu_u_to_oracle(inst, uh[b.u_off[i]:b.u_off[i] + _usize(inst)].astype(np.float64))
        x0o, zs, us = WS.receding_shift(inst, np.asarray(inst.x0, np.float32).astype(np.float64),
                                        zi, ui, w=w[xo])
        g = O.OracleGraph(W.mpc_graph(dataclasses.replace(inst, x0=x0o), box=inst.u_box > 0))
        g.set_state(zs, us)
        ko = g.run(20000, tol=1e-4)
        assert abs(int(itw[i]) - ko) <= max(2, 0.01 * ko), (i, itw[i], ko)
        zg = zwh[b.z_off[i]:b.z_off[i] + _zsize(inst)]
        assert rel(zg, g.z) < 1e-3, (i, rel(zg, g.z))
