"""GPU parity of the batched MPC solver against the FP64 oracle.

Each instance of the batch is compared with the oracle running the same
instance's factor graph (``workloads.mpc_graph``):
  * fixed iteration count: FP32 iterates within 1e-4 relative after 50
    iterations (every instance of a batch with the extreme shapes);
  * to tolerance 1e-4: same stopping iteration (+-2: FP32 vs FP64 residuals
    near the threshold) and z within 1e-4 relative;
  * dual completion: every edge's initial dual equals the oracle's;
  * warm start from the oracle's solution with dual completion stops after
    one iteration; the schedule (plan) never changes results (bitwise).
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import warmstart as WS
from tests.helpers import rel

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _mpc():
    from paper_1603_02526_amd import mpc as M
    return M


def _edge_instances():
    """Shapes at the edges of the solver's limits and of its lane mapping."""
    rng = np.random.default_rng(77)
    out = []
    for T, n, m, box in [(1, 4, 2, 1.0), (2, 1, 1, 1.0), (63, 12, 4, 1.0), (64, 5, 3, 1.0),
                         (65, 8, 2, 1.0), (128, 6, 4, 0.5), (129, 9, 3, 1.0), (200, 12, 4, 1.0),
                         (256, 4, 2, 1.0), (40, 7, 3, 0.0), (30, 3, 1, 1.0)]:
        A, B = W.mpc_system(rng, n, m)
        out.append(W.MPCInstance(T, n, m, A, B, rng.standard_normal(n) * 2, np.ones(n),
                                 np.full(m, 0.1), box))
    return out


def _solve(batch, insts, tol, max_iter, z_init=None, dual=False):
    x0 = torch.tensor(batch.pack_x0([i.x0 for i in insts]), device="cuda")
    z = torch.zeros(batch.z_total, dtype=torch.float32, device="cuda")
    it = torch.zeros(batch.n_inst, dtype=torch.int32, device="cuda")
    zi = None if z_init is None else torch.tensor(np.asarray(z_init, np.float32), device="cuda")
    batch.solve(x0, z, it, z_init=zi, dual=dual, tol=tol, max_iter=max_iter)
    torch.cuda.synchronize()
    return z.cpu().numpy().astype(np.float64), it.cpu().numpy()


def _oracle(inst, iters, tol=0.0, z0=None, u0=None):
    p = W.mpc_graph(inst, box=inst.u_box > 0)
    g = O.OracleGraph(p)
    if z0 is not None:
        g.set_state(z0, u0)
    k = g.run(iters, tol)
    return g.z, k


def test_fixed_iterations_parity_all_shapes():
    M = _mpc()
    insts = _edge_instances() + W.mpc_batch(20, seed=61)
    b = M.MPCBatch(insts)
    z, it = _solve(b, insts, tol=1e-30, max_iter=50)
    assert np.all(it == -50)
    for i, zi in enumerate(b.split_z(z)):
        zo, _ = _oracle(insts[i], 50)
        assert rel(zi, zo) < 1e-4, (i, insts[i].T, insts[i].n, insts[i].m, rel(zi, zo))


def test_to_tolerance_parity():
    M = _mpc()
    insts = W.mpc_batch(64, seed=62)
    b = M.MPCBatch(insts)
    z, it = _solve(b, insts, tol=1e-4, max_iter=10000)
    assert np.all(it > 0)
    order = np.argsort([i.T for i in insts])
    sample = list(order[:4]) + list(order[-4:]) + list(range(0, 64, 8))
    zs = b.split_z(z)
    for i in sorted(set(int(s) for s in sample)):
        zo, ko = _oracle(insts[i], 10000, tol=1e-4)
        assert abs(int(it[i]) - ko) <= 2, (i, it[i], ko)
        assert rel(zs[i], zo) < 1e-4, (i, rel(zs[i], zo))


def _gpu_u_to_oracle(inst, ug):
    """Per-step GPU dual layout [dx|du|dx1|qu|bx|qx] -> the oracle's edge order."""
    T, n, m = inst.T, inst.n, inst.m
    k = n + m
    st = ug.reshape(T, 3 * k)
    dx, du, dx1 = st[:, :n], st[:, n:n + m], st[:, n + m:2 * n + m]
    qu, bx, qx = st[:, 2 * n + m:2 * n + 2 * m], st[:, 2 * n + 2 * m:2 * n + 3 * m], st[:, 2 * n + 3 * m:]
    parts = [du[0], dx1[0]]
    for t in range(1, T):
        parts += [dx[t], du[t], dx1[t]]
    parts += list(qx) + list(qu)
    if inst.u_box > 0:
        parts += list(bx)
    return np.concatenate(parts)


def test_dual_completion_parity():
    M = _mpc()
    insts = _edge_instances()[:9] + W.mpc_batch(8, seed=63)
    b = M.MPCBatch(insts)
    rng = np.random.default_rng(4)
    z = rng.standard_normal(b.z_total).astype(np.float32)
    u = torch.zeros(b.u_total, dtype=torch.float32, device="cuda")
    b.dual_complete(torch.tensor(z, device="cuda"), u)
    torch.cuda.synchronize()
    u = u.cpu().numpy().astype(np.float64)
    for i, inst in enumerate(insts):
        o = b.z_off[i]
        zi = z[o:o + inst.T * (inst.n + inst.m)].astype(np.float64)
        uo = WS.dual_completion(inst, zi)
        ug = _gpu_u_to_oracle(inst, u[b.u_off[i]:b.u_off[i] + 3 * inst.T * (inst.n + inst.m)])
        assert rel(ug, uo) < 1e-5, (i, rel(ug, uo))


def test_warm_start_from_solution_stops_at_once():
    M = _mpc()
    insts = W.mpc_batch(12, seed=64, T_range=(20, 80))
    b = M.MPCBatch(insts)
    zstar = np.concatenate([_oracle(i, 200000, tol=1e-11)[0] for i in insts])
    z, it = _solve(b, insts, tol=1e-4, max_iter=10000, z_init=zstar, dual=True)
    assert np.all((it >= 1) & (it <= 2)), it
    # z alone (u0 = 0) does not give that
    z2, it2 = _solve(b, insts, tol=1e-4, max_iter=10000, z_init=zstar, dual=False)
    assert np.all(it2 > 5), it2


def test_plans_and_autotuner_do_not_change_results():
    M = _mpc()
    insts = W.mpc_batch(96, seed=65)
    b = M.MPCBatch(insts)
    ref_z, ref_it = _solve(b, insts, tol=1e-4, max_iter=10000)
    for pack, order, grid in [(1, 0, 0), (2, 2, 0), (4, 1, 7), (4, 2, 96)]:
        b.set_plan(pack, order, grid)
        z, it = _solve(b, insts, tol=1e-4, max_iter=10000)
        assert np.array_equal(z, ref_z) and np.array_equal(it, ref_it)
    x0 = torch.tensor(b.pack_x0([i.x0 for i in insts]), device="cuda")
    zs = torch.zeros(b.z_total, device="cuda")
    its = torch.zeros(b.n_inst, dtype=torch.int32, device="cuda")
    times = b.tune(x0, zs, its, tol=1e-4, reps=1)
    assert len(times) == 18 and all(t > 0 for t in times)
    z, it = _solve(b, insts, tol=1e-4, max_iter=10000)
    assert np.array_equal(z, ref_z) and np.array_equal(it, ref_it)
    # longest measured solve first (the tuning run recorded the iterations)
    for pack, grid in [(4, 0), (1, 96)]:
        b.set_plan(pack, 3, grid)
        z, it = _solve(b, insts, tol=1e-4, max_iter=10000)
        assert np.array_equal(z, ref_z) and np.array_equal(it, ref_it)


def test_max_iter_reported_negative():
    M = _mpc()
    insts = W.mpc_batch(5, seed=66)
    b = M.MPCBatch(insts)
    z, it = _solve(b, insts, tol=1e-4, max_iter=3)
    assert np.all(it == -3)


def test_nan_instance_is_reported_unconverged():
    """A NaN in one instance's x0 (one wavefront, and one of the lockstep
    instances) never meets the stopping rule: its count is -max_iter, and
    the other instances' results are those of a batch without it."""
    M = _mpc()
    insts = _edge_instances()[:6]
    bad = [1, 4]                      # T = 2 (one wavefront) and T = 65 (two lockstep)
    x0s = [i.x0.copy() for i in insts]
    for b in bad:
        x0s[b][0] = np.nan
    batch = M.MPCBatch(insts)
    x0 = torch.tensor(batch.pack_x0(x0s), device="cuda")
    z = torch.zeros(batch.z_total, dtype=torch.float32, device="cuda")
    it = torch.zeros(batch.n_inst, dtype=torch.int32, device="cuda")
    batch.solve(x0, z, it, tol=1e-4, max_iter=300)
    torch.cuda.synchronize()
    it = it.cpu().numpy()
    assert all(it[b] == -300 for b in bad)
    ref_z, ref_it = _solve(batch, insts, 1e-4, 300)
    zz = z.cpu().numpy()
    assert any(ref_it[k] > 0 for k in range(len(insts)) if k not in bad)
    for k in range(len(insts)):
        if k in bad:
            continue
        assert it[k] == ref_it[k]
        sl = batch.split_z(zz)[k]
        np.testing.assert_array_equal(sl, batch.split_z(ref_z.astype(np.float32))[k])


def test_full_batch_4096_sampled_against_oracle():
    """The benchmark's batch (4096 instances, seed 1003) in the launch
    configuration the benchmark times (the autotuned plan): every instance
    converges, and sampled instances (the slowest four and twelve seeded
    ones) match the oracle run to the same tolerance: stopping iteration
    within max(2, 1 %) (slowly converging instances cross the threshold at
    slightly different iterations in FP32 and FP64), stage cost within 1e-3
    relative and z within 1e-3 relative."""
    M = _mpc()
    insts = W.mpc_batch(4096, seed=1003)
    b = M.MPCBatch(insts)
    x0 = torch.tensor(b.pack_x0([i.x0 for i in insts]), device="cuda")
    zs = torch.zeros(b.z_total, device="cuda")
    its = torch.zeros(b.n_inst, dtype=torch.int32, device="cuda")
    b.tune(x0, zs, its, tol=1e-4, reps=1)
    z, it = _solve(b, insts, tol=1e-4, max_iter=10000)
    assert np.all(it > 0), np.sum(it <= 0)
    rng = np.random.default_rng(5)
    sample = list(np.argsort(-it)[:4]) + list(rng.choice(4096, 12, replace=False))
    zsplit = b.split_z(z)
    for i in sorted(set(int(s) for s in sample)):
        inst = insts[i]
        zo, ko = _oracle(inst, 20000, tol=1e-4)
        assert abs(int(it[i]) - ko) <= max(2, 0.01 * ko), (i, it[i], ko)
        co = O.mpc_objective(inst, zo)["cost"]
        cg = O.mpc_objective(inst, zsplit[i])["cost"]
        assert abs(cg - co) <= 1e-3 * abs(co), (i, cg, co)
        assert rel(zsplit[i], zo) < 1e-3, (i, rel(zsplit[i], zo))


def test_short_horizon_batch_on_128_thread_workgroups():
    """A batch whose instances all have T <= 128 runs on 128-thread
    workgroups (twice as many resident).  Its results equal, bit for bit,
    those of the same instances in a batch that also holds a T = 200
    instance (256-thread workgroups), under every packing, and match the
    oracle after 50 iterations."""
    M = _mpc()
    short = W.mpc_batch(40, seed=67, T_range=(20, 128))
    rng = np.random.default_rng(68)
    A_, B_ = W.mpc_system(rng, 6, 2)
    long_ = W.MPCInstance(200, 6, 2, A_, B_, rng.standard_normal(6), np.ones(6),
                          np.full(2, 0.1), 1.0)
    a = M.MPCBatch(short)
    b = M.MPCBatch(short + [long_])
    assert a.plan()["resident"] > b.plan()["resident"]
    za, ia = _solve(a, short, tol=1e-4, max_iter=10000)
    zb, ib = _solve(b, short + [long_], tol=1e-4, max_iter=10000)
    assert np.array_equal(ia, ib[:-1])
    assert np.array_equal(za, zb[:a.z_total])
    for pack in (4, 2, 1):
        a.set_plan(pack, 1, 0)
        z2, i2 = _solve(a, short, tol=1e-4, max_iter=10000)
        assert np.array_equal(z2, za) and np.array_equal(i2, ia)
    z50, _ = _solve(a, short, tol=1e-30, max_iter=50)
    for i in range(0, 40, 5):
        zo, _ = _oracle(short[i], 50)
        zi = z50[a.z_off[i]:a.z_off[i] + short[i].T * (short[i].n + short[i].m)]
        assert rel(zi, zo) < 1e-4, (i, rel(zi, zo))
