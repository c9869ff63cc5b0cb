"""GPU parity of the paper's own SVM graph (Sec. V-C, App. C): a copy w_i
of the weight vector per point tied by equality factors, one margin and one
minimal-error factor per point and a 1/N-weighted norm factor per copy.

Bars as for the other graphs: FP64 kernels within 1e-9 of the oracle, FP32
within 1e-4 after 50 iterations, one step from a common state element by
element (with residuals and the zero dual sums), both drivers, general
alpha, and the converged classifier against the oracle's.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1603_02526_amd import admm as A
from tests.helpers import rel
from tests.test_gpu_graph import _check, _one_step, _pair, _traj

pytestmark = pytest.mark.gpu

FP32, FP64 = A.FP32, A.FP64


@pytest.mark.parametrize("N,d", [(300, 5), (257, 20), (130, 40), (2, 3)])
@pytest.mark.parametrize("prec,iters,tol", [(FP64, 60, 1e-9), (FP32, 50, 1e-4)])
def test_copies_parity(N, d, prec, iters, tol):
    p = W.svm_copies(N, d, seed=91 + N)
    g, o = _traj(p, iters, prec, tol, driver=A.DRIVER_LAUNCHES)
    assert g.info()["driver"] == A.DRIVER_LAUNCHES
    _one_step(p, 40, prec, 1e-12 if prec == FP64 else 1e-5, driver=A.DRIVER_LAUNCHES)


@pytest.mark.parametrize("N,d,seed,iters", [(60, 100, 613, 40), (40, 200, 614, 30)])
@pytest.mark.parametrize("prec,tol", [(FP64, 1e-9), (FP32, 1e-4)])
def test_copies_wide_parity(N, d, seed, iters, prec, tol):
    """Margin factors with d > 64 (two-sweep path)."""
    p = W.svm_copies(N, d, seed=seed)
    _traj(p, iters, prec, tol, driver=A.DRIVER_LAUNCHES)
    _one_step(p, 20, prec, 1e-12 if prec == FP64 else 1e-5, driver=A.DRIVER_LAUNCHES)


@pytest.mark.parametrize("prec,iters,tol", [(FP64, 60, 1e-9), (FP32, 30, 1e-4)])
def test_copies_resident_driver(prec, iters, tol):
    p = W.svm_copies(40, 3, seed=95)
    g, o = _traj(p, iters, prec, tol, driver=A.DRIVER_RESIDENT)
    assert g.info()["driver"] == A.DRIVER_RESIDENT
    _one_step(p, 20, prec, 1e-12 if prec == FP64 else 1e-5, driver=A.DRIVER_RESIDENT)


@pytest.mark.parametrize("alpha", [1.5, 0.7])
def test_copies_general_alpha_fp64(alpha):
    p = W.svm_copies(150, 4, seed=96)
    _traj(p, 30, FP64, 1e-9, alpha=alpha)


def test_copies_converged_classifier_fp32():
    """Run to convergence in FP32: every copy and b agree with the oracle's
    converged solution (the hinge graph's optimum), and the objective
    1/2 |w|^2 + sum max(0, 1 - y(w.a + b)) agrees within 1e-3."""
    N, d = 12, 3
    p = W.svm_copies(N, d, seed=97, sep=1.0)
    g = A.Graph.from_problem(p, precision=FP32)
    g.run(6000)
    o = O.OracleGraph(p)
    o.run(400000, tol=1e-13)
    zg, zo = g.z(), o.z
    for i in range(N):
        assert rel(zg[i * d:(i + 1) * d], zo[:d]) < 1e-3
    assert abs(zg[N * d] - zo[N * d]) < 1e-3

    def objective(z):
        w, b = z[:d], z[N * d]
        a, y = p.meta["a"], p.meta["y"]
        return 0.5 * w @ w + np.sum(np.maximum(0.0, 1.0 - y * (a @ w + b)))
    fo = objective(zo)
    assert abs(objective(zg) - fo) <= 1e-3 * abs(fo)


@pytest.mark.parametrize("prec,tol", [(FP64, 1e-9), (FP32, 1e-4)])
def test_margin_with_two_biases(prec, tol):
    """Half the points use a second bias variable, so the margin bucket's b
    edge is not one shared variable and every factor contributes its own m
    (the per-workgroup partial applies only to a shared bias)."""
    import dataclasses
    N, d = 300, 4
    p = W.svm_copies(N, d, seed=98)
    g0 = p.groups[0]
    vid = g0.var_ids.copy()
    extra = p.n_vars
    vid[N // 2:, 1] = extra
    groups = [W.FactorGroup("margin", vid, g0.params)] + p.groups[1:]
    q = dataclasses.replace(p, var_dims=np.append(p.var_dims, 1).astype(np.int32),
                            groups=groups, z0=np.zeros(p.n_scalars + 1))
    _traj(q, 50, prec, tol)
    _one_step(q, 30, prec, 1e-12 if prec == FP64 else 1e-5)
