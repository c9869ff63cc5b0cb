"""GPU parity of the three-weight variant (Sec. II: per-edge weights with an
improved update scheme; every message weight is 0 or rho) against the
oracle's, on packing graphs: dense pair tiles with the sparse pair state
(FP32) and the general layout (FP32 and FP64), launches and graph blocks,
element by element with the oracle's own per-entry sensitivity."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1603_02526_amd import admm as A
from tests import parity as P
from tests.helpers import slot_z

pytestmark = pytest.mark.gpu

FP32, FP64 = A.FP32, A.FP64


def _eps(prec):
    return 1e-16 if prec == FP64 else 6e-8


def _graph(p, prec, dense=False, driver=A.DRIVER_AUTO):
    return A.Graph.from_problem(p, precision=prec, three_weight=True, driver=driver,
                                pair_state=A.PAIR_STATE_DENSE if dense else A.PAIR_STATE_AUTO)


def _check(g, o, tol, sens):
    P.check(P.errors(g.z(), g.u(), g.x(), o.z, o.u, o.x, o.slot_z, sens, tol), tol)


CASES = {
    "tri10": lambda: W.workload("packing_tri10"),
    "sq65": lambda: W.packing(65, "square", 0.3 / np.sqrt(65), seed=3),
    "sq200": lambda: W.packing(200, "square", 0.3 / np.sqrt(200), seed=4),
    "tri130": lambda: W.packing(130, "triangle", 0.3 / np.sqrt(130), seed=7),
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec,dense,iters,tol", [(FP64, False, 12, 1e-9),
                                                  (FP32, False, 8, 1e-4),
                                                  (FP32, True, 8, 1e-4)])
def test_twa_trajectory(name, prec, dense, iters, tol):
    p = CASES[name]()
    g = _graph(p, prec, dense)
    inf = g.info()
    assert inf["three_weight"] == 1
    if prec == FP32 and not dense:
        assert inf["n_pair_tiles"] > 0 and inf["sparse_pair_state"] == 1
    else:
        assert inf["n_pair_tiles"] == 0
    worst, sens = P.sensitivity(p, iters, _eps(prec), twa=True)
    assert P.norm_part(worst) < tol / 20, worst
    o = O.OracleGraph(p, twa=True)
    g.run(iters)
    o.run(iters)
    _check(g, o, tol, sens)
    (r, s), (ro, so) = g.residuals(), o.residuals()
    zmax = np.max(np.abs(o.z)) + 1.0
    assert abs(r - ro) <= tol * zmax and abs(s - so) <= tol * zmax, (r, ro, s, so)
    # edges that sent weight 0 in the last iteration end with u = 0 exactly
    u = g.u()
    assert np.all(u[o.wr == 0.0] == 0.0)


@pytest.mark.parametrize("dense", [False, True])
def test_twa_one_step_full_size(dense):
    """2000 disks: a few steps from a common state against the oracle."""
    p = W.workload("packing_sq2000")
    g = _graph(p, FP32, dense)
    g.run(20)
    z, u = g.z(), g.u()
    g.set_state(z, u)
    o = O.OracleGraph(p, twa=True)
    o.set_state(z, u)
    g.run(3)
    o.run(3)
    _, sens = P.sensitivity(p, 3, _eps(FP32), z0=z, u0=u, twa=True)
    _check(g, o, 1e-5, sens)


def test_twa_final_objective_tri10():
    """The 10-disk benchmark packing to 2000 iterations in FP32: objective and
    feasibility against the FP64 oracle's run of the same variant."""
    p = W.workload("packing_tri10")
    g = _graph(p, FP32)
    g.run(2000)
    o = O.OracleGraph(p, twa=True)
    o.run(2000)
    fg, fo = O.packing_objective(p, g.z()), O.packing_objective(p, o.z)
    assert abs(fg["objective"] - fo["objective"]) <= 1e-3 * abs(fo["objective"])
    assert fg["max_violation"] < 1e-5 and fo["max_violation"] < 1e-5


@pytest.mark.parametrize("dense", [False, True])
def test_twa_split_runs_graph_driver_and_determinism(dense):
    p = W.packing(150, "square", 0.04, seed=12)
    a = _graph(p, FP32, dense, driver=A.DRIVER_LAUNCHES)
    a.run(37)
    b = _graph(p, FP32, dense)
    assert b.info()["driver"] == A.DRIVER_GRAPH
    b.run(20)
    b.run(17)
    c = _graph(p, FP32, dense)
    c.run(37)
    for q in (b, c):
        assert np.array_equal(a.z(), q.z()) and np.array_equal(a.u(), q.u())
        assert np.array_equal(a.x(), q.x())
    a.set_state(p.z0)
    c.set_state(p.z0)
    a.run(64)
    c.run(64)
    assert np.array_equal(a.z(), c.z()) and np.array_equal(a.u(), c.u())


def test_twa_unsupported_graphs():
    for q in (W.svm(300, 3, seed=1), W.mpc_graph(W.mpc_batch(1, seed=41)[0])):
        with pytest.raises(A.AdmmError) as e:
            A.Graph.from_problem(q, three_weight=True)
        assert e.value.status == A.E_UNSUPPORTED
    with pytest.raises(A.AdmmError) as e:
        A.Graph.from_problem(W.workload("packing_tri10"), three_weight=True, alpha=1.5)
    assert e.value.status == A.E_UNSUPPORTED
