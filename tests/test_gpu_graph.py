"""GPU parity of the factor-graph engine against the FP64 oracle.

Same seeded inputs on both sides (``workloads``).  Bars:
  * FP64 instantiation of the kernels: iterates within 1e-9 relative;
  * FP32: iterates (z, u, x) within 1e-4 relative after 50 iterations and
    the final objective within 1e-3 relative;
  * bitwise run-to-run determinism and split-run (resume) equivalence.
Full-size graphs are checked on one iteration from a common state (the
oracle can afford one iteration at 2000 disks) and on invariants that hold
at any size.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from paper_1603_02526_amd import admm as A
from tests import parity as P
from tests.helpers import rel, slot_z

pytestmark = pytest.mark.gpu

FP32, FP64 = A.FP32, A.FP64


def _pair(problem, iters, precision, alpha=None, u0=None, pair_rows=0, driver=A.DRIVER_AUTO):
    g = A.Graph.from_problem(problem, precision=precision, alpha=alpha, pair_rows=pair_rows,
                             driver=driver)
    o = O.OracleGraph(problem, alpha=alpha)
    if u0 is not None:
        g.set_state(problem.z0, u0)
        o.set_state(problem.z0, u0)
    g.run(iters)
    o.run(iters)
    return g, o


def _check(g, o, tol, sens=None):
    """z, u and x against the oracle, as a relative norm and element by
    element (tests/parity.py: z relative to |z|; u and x relative to the
    size of the operands they are formed from, since u = m - z cancels and
    its error scales with |z_b|, not |u|; per-entry allowance for the
    entries the oracle itself cannot resolve to tol/20 left to the norm when
    `sens` is given)."""
    e = P.errors(g.z(), g.u(), g.x(), o.z, o.u, o.x, o.slot_z, sens, tol)
    P.check(e, tol)
    return e


def _eps(prec):
    return 1e-16 if prec == FP64 else 6e-8


def _well_conditioned(problem, iters, prec, tol, alpha=None, u0=None):
    """Trajectory parity is asserted only where the oracle's own trajectory,
    under rounding-size noise on z and u every iteration, moves far less
    than the tolerance in norm (below tol/20).  Returns the per-entry
    sensitivities for the element-wise bound.  Packing from overlapping
    random starts is chaotic, so these horizons are short there."""
    worst, sens = P.sensitivity(problem, iters, _eps(prec), alpha, u0=u0)
    assert P.norm_part(worst) < tol / 20, f"test case ill-conditioned: oracle self-sensitivity {worst}"
    return sens


def _traj(problem, iters, prec, tol, alpha=None, u0=None, pair_rows=0, driver=A.DRIVER_AUTO):
    sens = _well_conditioned(problem, iters, prec, tol, alpha, u0)
    g, o = _pair(problem, iters, prec, alpha=alpha, u0=u0, pair_rows=pair_rows, driver=driver)
    _check(g, o, tol, sens)
    return g, o


@pytest.mark.parametrize("prec,iters,tol", [(FP64, 300, 1e-9), (FP32, 50, 1e-4)])
def test_packing_triangle_10(prec, iters, tol):
    p = W.workload("packing_tri10")
    g, o = _traj(p, iters, prec, tol)
    r, s = g.residuals()
    ro, so = o.residuals()
    assert abs(r - ro) <= 1e-6 * max(ro, 1e-12) + (1e-12 if prec == FP64 else 1e-5)
    assert abs(s - so) <= 1e-6 * max(so, 1e-12) + (1e-12 if prec == FP64 else 1e-5)


def test_packing_triangle_10_final_objective_fp32():
    p = W.workload("packing_tri10")
    g, o = _pair(p, 2000, FP32)
    fg = O.packing_objective(p, g.z())
    fo = O.packing_objective(p, o.z)
    assert abs(fg["objective"] - fo["objective"]) <= 1e-3 * abs(fo["objective"])
    assert fg["max_violation"] < 1e-3


@pytest.mark.parametrize("rb", [16, 32, 64])
@pytest.mark.parametrize("N,shape,seed", [(2, "square", 1), (65, "square", 3),
                                          (130, "triangle", 7), (200, "square", 4)])
def test_packing_tiles_ragged_fp64(N, shape, seed, rb):
    p = W.packing(N, shape, 0.3 / np.sqrt(N), seed=seed)
    g, o = _traj(p, 12, FP64, 1e-9, pair_rows=rb, driver=A.DRIVER_LAUNCHES)
    assert g.info()["n_pair_tiles"] == len({(i // rb, j // 64) for i in range(N)
                                            for j in range(i + 1, N)})
    _one_step(p, 40, FP64, 1e-12, pair_rows=rb, driver=A.DRIVER_LAUNCHES)


@pytest.mark.parametrize("rb", [16, 32, 64])
@pytest.mark.parametrize("N,shape,seed", [(2, "square", 1), (65, "square", 3),
                                          (130, "triangle", 7), (200, "square", 4)])
def test_packing_tiles_ragged_fp32(N, shape, seed, rb):
    """FP32 with alpha = 1 takes the 16-byte tile path: one step from a common
    state against the oracle, including residuals and x, on ragged sizes."""
    p = W.packing(N, shape, 0.3 / np.sqrt(N), seed=seed)
    _one_step(p, 40, FP32, 1e-5, pair_rows=rb, driver=A.DRIVER_LAUNCHES)
    g = A.Graph.from_problem(p, pair_rows=rb, driver=A.DRIVER_LAUNCHES)
    assert g.info()["n_pair_tiles"] == len({(i // rb, j // 64) for i in range(N)
                                            for j in range(i + 1, N)})


@pytest.mark.parametrize("N,seed,iters", [(65, 12, 8), (200, 12, 8)])
def test_packing_tiles_fp32(N, seed, iters):
    """Overlapping random disks: after ten iterations the oracle's own u and
    x move by 6e-6 to 9e-6 (relative norm, the largest of four noisy runs)
    under rounding-size noise, above the tol/20 precondition; eight keep
    it below."""
    p = W.packing(N, "square", 0.3 / np.sqrt(N), seed=seed)
    _traj(p, iters, FP32, 1e-4)
    _one_step(p, 40, FP32, 1e-5)


@pytest.mark.parametrize("alpha", [1.5, 0.8])
def test_general_alpha_fp64(alpha):
    p = W.packing(30, "triangle", 0.1, seed=7)
    _traj(p, 30, FP64, 1e-9, alpha=alpha)
    _one_step(p, 40, FP64, 1e-12, alpha=alpha)
    p = W.svm(700, 5, seed=8)
    _traj(p, 60, FP64, 1e-9, alpha=alpha)


def test_nonzero_initial_u_fp64():
    p = W.packing(40, "square", 0.08, seed=9)
    u0 = np.random.default_rng(5).standard_normal(p.n_slots) * 0.01
    _traj(p, 15, FP64, 1e-9, u0=u0)


def test_general_pair_layouts_fp64():
    """Incomplete and reversed pair lists go through the general layout."""
    p = W.packing(50, "square", 0.07, seed=10)
    g0 = p.groups[0]
    keep = np.random.default_rng(1).random(g0.n) < 0.7
    vid = g0.var_ids[keep].copy()
    vid[::3] = vid[::3][:, [2, 3, 0, 1]]
    p.groups[0] = W.FactorGroup("nonoverlap", vid, g0.params, True)
    g, o = _traj(p, 12, FP64, 1e-9)
    assert g.info()["n_pair_tiles"] == 0
    _one_step(p, 40, FP64, 1e-12)
    _one_step(p, 40, FP32, 1e-5)


@pytest.mark.parametrize("N,d,prec,iters,tol", [(3000, 20, FP64, 100, 1e-9),
                                                (3000, 20, FP32, 50, 1e-4),
                                                (777, 40, FP64, 50, 1e-9),
                                                (300, 3, FP32, 50, 1e-4)])
def test_svm_parity(N, d, prec, iters, tol):
    p = W.svm(N, d, seed=11 + N)
    _traj(p, iters, prec, tol)


@pytest.mark.parametrize("d", [1, 6, 13, 24, 31, 32])
def test_svm_four_lane_hinge(d):
    """FP32 shared-variable hinge with four lanes per four factors: every
    register width (2, 4, 6 and 8 edges per lane), a factor count that is not
    a multiple of 4 or of the workgroup (1001), and d = 32, which keeps two
    lanes per factor (one partial per variable per workgroup: 256 factors per
    workgroup, 128 at d = 32)."""
    p = W.svm(1001, d, seed=700 + d)
    g = A.Graph.from_problem(p, precision=FP32, driver=A.DRIVER_LAUNCHES)
    per_wg = 128 if d == 32 else 256
    assert g.info()["n_contributions"] == -(-1001 // per_wg) * (d + 1) + d
    _traj(p, 50, FP32, 1e-4, driver=A.DRIVER_LAUNCHES)
    _one_step(p, 20, FP32, 1e-5, driver=A.DRIVER_LAUNCHES)


@pytest.mark.parametrize("N,d,seed,prec,iters,tol", [(500, 100, 611, FP64, 50, 1e-9),
                                                     (500, 100, 611, FP32, 50, 1e-4),
                                                     (400, 200, 612, FP64, 40, 1e-9),
                                                     (400, 200, 612, FP32, 40, 1e-4)])
def test_svm_wide_parity(N, d, seed, prec, iters, tol):
    """d > 64 weights (the paper's dimension sweep reaches 200): the hinge
    takes the two-sweep path without register arrays."""
    p = W.svm(N, d, seed=seed)
    _traj(p, iters, prec, tol, driver=A.DRIVER_LAUNCHES)
    _one_step(p, 20, prec, 1e-12 if prec == FP64 else 1e-5, driver=A.DRIVER_LAUNCHES)


def test_svm_wide_resident_fp32():
    """The two-sweep hinge inside the resident driver (in FP64 a d > 64
    hinge bucket does not fit the LDS image: (2(d+1) + d+3) x 64 x 8 B)."""
    p = W.svm(24, 66, seed=615)
    g, o = _traj(p, 40, FP32, 1e-4, driver=A.DRIVER_RESIDENT)
    assert g.info()["driver"] == A.DRIVER_RESIDENT


def test_svm_nonuniform_hinge_fp64():
    """Hinge factors with different variable lists (two w copies)."""
    p = W.svm(500, 4, seed=21)
    hg = p.groups[0]
    vid = hg.var_ids.copy()
    vid[1::2, :4] += 5          # odd points use a second copy of w
    dims = np.ones(10, np.int32)
    groups = [W.FactorGroup("hinge", vid, hg.params),
              W.FactorGroup("l2", np.arange(4, dtype=np.int32)[None, :], np.array([1.0]), True),
              W.FactorGroup("l2", np.arange(5, 9, dtype=np.int32)[None, :], np.array([1.0]), True)]
    q = W.Problem("svm2", dims, groups, np.zeros(10))
    g, o = _pair(q, 60, FP64)
    _check(g, o, 1e-9)


def test_svm_final_objective_fp32():
    p = W.svm(20000, 20, seed=31)
    g, o = _pair(p, 500, FP32)
    fg, fo = O.svm_objective(p, g.z()), O.svm_objective(p, o.z)
    assert abs(fg - fo) <= 1e-3 * abs(fo)


@pytest.mark.parametrize("seed", [41, 42])
def test_mpc_graph_parity(seed):
    inst = W.mpc_batch(1, seed=seed)[0]
    p = W.mpc_graph(inst)
    _traj(p, 80, FP64, 1e-9)
    _traj(p, 50, FP32, 1e-4)


def test_degenerate_graphs():
    # a variable with no edge keeps its z; a single disk has no pair bucket
    p = W.packing(1, "square", 0.2, seed=3)
    dims = np.array([2, 1, 3], np.int32)
    q = W.Problem("iso", dims, p.groups, np.r_[p.z0, [7.0, 8.0, 9.0]])
    g, o = _pair(q, 30, FP64)
    _check(g, o, 1e-9)
    np.testing.assert_array_equal(g.z()[3:], [7.0, 8.0, 9.0])
    # no factors at all
    g = A.Graph([2, 1])
    g.finalize(0)
    g.set_state(np.array([1.0, 2.0, 3.0]))
    g.run(5)
    np.testing.assert_array_equal(g.z(), [1.0, 2.0, 3.0])
    # zero iterations
    g = A.Graph.from_problem(W.workload("packing_tri10"))
    g.run(0)
    np.testing.assert_array_equal(g.z(), W.workload("packing_tri10").z0.astype(np.float32))


@pytest.mark.parametrize("case", ["packing_tri10", "packing_200", "svm", "mpc"])
@pytest.mark.parametrize("bad", [np.nan, np.inf])
def test_nonfinite_state_reported(case, bad):
    """A NaN or infinity set from the host reaches the residuals of the run,
    which report ADMM_E_NUMERIC; the status stays until a new state is
    imported (every layout: resident driver, sparse pair tiles, shared
    hinge, linear dynamics)."""
    p = {"packing_tri10": lambda: W.workload("packing_tri10"),
         "packing_200": lambda: W.packing(200, "square", 0.02, seed=47),
         "svm": lambda: W.svm(3000, 20, seed=13),
         "mpc": lambda: W.mpc_graph(W.mpc_batch(1, seed=41)[0])}[case]()
    g = A.Graph.from_problem(p)
    z0 = np.array(p.z0, dtype=np.float64)
    z0[len(z0) // 2] = bad
    g.set_state(z0)
    g.run(5)
    for _ in range(2):
        with pytest.raises(A.AdmmError) as e:
            g.residuals()
        assert e.value.status == A.E_NUMERIC
    g.set_state(p.z0)
    g.run(5)
    r, s = g.residuals()
    assert np.isfinite(r) and np.isfinite(s)


def test_determinism_and_resume():
    p = W.packing(150, "square", 0.04, seed=12)
    a = A.Graph.from_problem(p)
    a.run(37)
    b = A.Graph.from_problem(p)
    b.run(37)
    assert np.array_equal(a.z(), b.z()) and np.array_equal(a.u(), b.u())
    c = A.Graph.from_problem(p)
    c.run(20)
    c.run(17)
    assert np.array_equal(a.z(), c.z()) and np.array_equal(a.u(), c.u())
    # profiled runs compute the same iterates
    d = A.Graph.from_problem(p)
    xm, zm = d.run_profiled(37)
    assert xm > 0 and zm > 0
    assert np.array_equal(a.z(), d.z())


@pytest.mark.parametrize("case,block", [("packing", 2), ("packing", 8), ("packing", 32),
                                        ("svm", 32), ("mpc", 4)])
def test_graph_driver_matches_launches(case, block):
    """Recorded iteration blocks run the same kernels in the same order as
    direct launches: identical bits after every run, with state reads,
    state imports and synchronisations between the replays, runs shorter
    than a block, and replays starting from either z buffer."""
    p = {"packing": lambda: W.packing(150, "square", 0.04, seed=12),
         "svm": lambda: W.svm(3000, 20, seed=13),
         "mpc": lambda: W.mpc_graph(W.mpc_batch(1, seed=41)[0])}[case]()
    a = A.Graph.from_problem(p, driver=A.DRIVER_LAUNCHES)
    b = A.Graph.from_problem(p, driver=A.DRIVER_GRAPH, graph_block=block)
    assert b.info()["driver"] == A.DRIVER_GRAPH
    for iters in (37, 1, 64, 3, 100, 2 * block + 1):
        a.run(iters)
        b.run(iters)
        assert np.array_equal(a.z(), b.z()) and np.array_equal(a.u(), b.u())
        assert np.array_equal(a.x(), b.x()) and a.residuals() == b.residuals()
    a.set_state(p.z0)
    b.set_state(p.z0)
    a.run(70)
    b.run(70)
    assert np.array_equal(a.z(), b.z()) and np.array_equal(a.u(), b.u())


def test_graph_driver_full_size_packing():
    p = W.workload("packing_sq2000")
    a = A.Graph.from_problem(p, driver=A.DRIVER_LAUNCHES)
    b = A.Graph.from_problem(p)
    assert b.info()["driver"] == A.DRIVER_GRAPH
    a.run(101)
    b.run(101)
    assert np.array_equal(a.z(), b.z()) and np.array_equal(a.u(), b.u())


def _one_step(problem, warm_iters, prec, tol, alpha=None, pair_rows=0, driver=A.DRIVER_AUTO,
              steps=1, pair_state=A.PAIR_STATE_AUTO):
    """Run the GPU warm_iters iterations, hand its (z, u) to both sides and
    compare `steps` further iterations element by element (one or a few
    steps: no trajectory sensitivity involved; from the second step on, the
    sparse pair state takes unmoved pairs' m from the previous z), then
    check that the duals around every variable sum to zero (Algorithm 2
    with u0 = 0 keeps that at any size)."""
    g = A.Graph.from_problem(problem, precision=prec, alpha=alpha, pair_rows=pair_rows,
                             driver=driver, pair_state=pair_state)
    g.run(warm_iters)
    z, u = g.z(), g.u()
    g.set_state(z, u)
    o = O.OracleGraph(problem, alpha=alpha)
    o.set_state(z, u)
    g.run(steps)
    o.run(steps)
    _, sens = P.sensitivity(problem, steps, _eps(prec), alpha, z0=z, u0=u)
    _check(g, o, tol, sens)
    # r = max_e |x_e - z_b(e)|: the kernel's maximum equals the one of its
    # own exported iterates, and against the oracle's r the bar is the
    # iterates' own (tolerance at the scale of z plus, at the entries
    # attaining either maximum, the allowance for what rounding alone moves
    # them in the oracle)
    (r, s), (ro, so) = g.residuals(), o.residuals()
    zmax = np.max(np.abs(o.z)) + 1.0
    sz = slot_z(problem)
    dg = np.abs(g.x() - g.z()[sz])
    assert abs(r - dg.max()) <= 1e-6 * dg.max() + (1e-12 if prec == FP64 else 1e-7), (r, dg.max())
    sx = sens["x"] + sens["z"][sz]
    ar = P.K_SENS * (sx[np.argmax(dg)] + sx[np.argmax(np.abs(o.x - o.z[sz]))])
    az = 2 * P.K_SENS * float(np.max(sens["z"], initial=0.0))
    assert abs(r - ro) <= tol * zmax + ar and abs(s - so) <= tol * zmax + az, (r, ro, s, so, ar, az)
    us = np.bincount(sz, weights=g.u(), minlength=problem.n_scalars)
    zz = g.z()
    scale = np.bincount(sz, weights=np.abs(g.u()) + np.abs(zz[sz]),
                        minlength=problem.n_scalars) + 1e-30
    assert np.max(np.abs(us) / scale) < (1e-12 if prec == FP64 else 1e-5)


@pytest.mark.parametrize("rb", [16, 32, 64])
def test_full_size_packing_2000_one_step(rb):
    _one_step(W.workload("packing_sq2000"), 20, FP32, 1e-5, pair_rows=rb)


@pytest.mark.parametrize("pair_state", [A.PAIR_STATE_AUTO, A.PAIR_STATE_DENSE])
def test_full_size_packing_2000_three_steps(pair_state):
    p = W.workload("packing_sq2000")
    g = A.Graph.from_problem(p, pair_state=pair_state)
    assert g.info()["sparse_pair_state"] == (1 if pair_state == A.PAIR_STATE_AUTO else 0)
    _one_step(p, 20, FP32, 1e-5, steps=3, pair_state=pair_state)


@pytest.mark.parametrize("N,shape,seed", [(2, "square", 1), (65, "square", 3),
                                          (130, "triangle", 7), (200, "square", 4)])
def test_sparse_pair_state_matches_dense(N, shape, seed):
    """Sparse and dense pair state compute the same iteration (unmoved pairs
    end at m = z exactly instead of (z - u) + u).  From the same start the
    two FP32 trajectories differ by rounding per iteration, which disks in
    contact amplify over eight iterations to ~1e-5: the cross-check bar is
    1e-4.  The element-wise bar is the oracle's, from a common state over
    four steps (the steps after the first use the implicit m)."""
    p = W.packing(N, shape, 0.3 / np.sqrt(N), seed=seed)
    gs = A.Graph.from_problem(p, driver=A.DRIVER_LAUNCHES)
    gd = A.Graph.from_problem(p, driver=A.DRIVER_LAUNCHES, pair_state=A.PAIR_STATE_DENSE)
    assert gs.info()["sparse_pair_state"] == 1 and gd.info()["sparse_pair_state"] == 0
    gs.run(8)
    gd.run(8)
    assert rel(gs.z(), gd.z()) < 1e-4 and rel(gs.x(), gd.x()) < 1e-4
    for st in (A.PAIR_STATE_AUTO, A.PAIR_STATE_DENSE):
        _one_step(p, 30, FP32, 1e-5, steps=4, driver=A.DRIVER_LAUNCHES, pair_state=st)


def test_full_size_svm_100k_one_step():
    _one_step(W.workload("svm_100k_d20"), 20, FP32, 1e-5)


def test_full_size_packing_2000_fp64_iterates():
    p = W.workload("packing_sq2000")
    g, o = _pair(p, 3, FP64)
    _check(g, o, 1e-9, P.sensitivity(p, 3, _eps(FP64))[1])
    _one_step(p, 30, FP64, 1e-12)


# ---------------------------------------------------------------------------
# Resident driver: the whole run in one workgroup with the state in LDS.
# ---------------------------------------------------------------------------
def _small_cases():
    inst = W.mpc_batch(1, seed=44)[0]
    inst.T = 12
    return {
        "packing_tri10": W.workload("packing_tri10"),
        "packing_2": W.packing(2, "square", 0.2, seed=1),
        "packing_12_general_pairs": W.packing(12, "square", 0.12, seed=2),
        "svm_300_d3": W.svm(300, 3, seed=311),
        "mpc_T12": W.mpc_graph(inst),
    }


@pytest.mark.parametrize("name", ["packing_tri10", "packing_2", "svm_300_d3", "mpc_T12"])
@pytest.mark.parametrize("prec,iters,tol", [(FP64, 60, 1e-9), (FP32, 30, 1e-4)])
def test_resident_driver_parity(name, prec, iters, tol):
    p = _small_cases()[name]
    g, o = _traj(p, iters, prec, tol, driver=A.DRIVER_RESIDENT)
    inf = g.info()
    assert inf["driver"] == A.DRIVER_RESIDENT and inf["n_pair_tiles"] == 0
    assert 0 < inf["resident_lds_bytes"] <= 96 * 1024
    r, s = g.residuals()
    ro, so = o.residuals()
    small = 1e-12 if prec == FP64 else 1e-5
    assert abs(r - ro) <= 1e-6 * max(ro, 1e-12) + small
    assert abs(s - so) <= 1e-6 * max(so, 1e-12) + small


@pytest.mark.parametrize("alpha", [1.0, 1.5])
def test_resident_driver_alpha_and_u0_fp64(alpha):
    p = _small_cases()["packing_12_general_pairs"]
    u0 = np.random.default_rng(6).standard_normal(p.n_slots) * 0.01
    g, o = _traj(p, 25, FP64, 1e-9, alpha=alpha, u0=u0, driver=A.DRIVER_RESIDENT)
    assert g.info()["driver"] == A.DRIVER_RESIDENT
    _one_step(p, 30, FP64, 1e-12, alpha=alpha, driver=A.DRIVER_RESIDENT)


@pytest.mark.parametrize("name", ["svm_300_d3", "mpc_T12"])
def test_resident_matches_launches(name):
    """Without pair tiles both drivers run the same arithmetic: the same
    iterates up to the order of the per-workgroup sums (the FP32 SVM's
    hinge takes two lanes per factor in a resident plan and four lanes per
    four factors otherwise).  Residuals are maxima of differences of
    z-sized values, so their error is bounded by the iterates' error times
    the size of z."""
    p = _small_cases()[name]
    for prec, tol in ((FP64, 1e-13), (FP32, 1e-6)):
        a = A.Graph.from_problem(p, precision=prec, driver=A.DRIVER_RESIDENT)
        b = A.Graph.from_problem(p, precision=prec, driver=A.DRIVER_LAUNCHES)
        assert a.info()["driver"] == A.DRIVER_RESIDENT
        assert b.info()["driver"] == A.DRIVER_LAUNCHES
        a.run(40)
        b.run(40)
        assert rel(a.z(), b.z()) <= tol and rel(a.u(), b.u()) <= tol and rel(a.x(), b.x()) <= tol
        zmax = float(np.max(np.abs(b.z()))) + 1.0
        for ra, rb_ in zip(a.residuals(), b.residuals()):
            assert abs(ra - rb_) <= 4 * tol * zmax, (ra, rb_)


def test_resident_determinism_resume_and_profiled():
    p = W.workload("packing_tri10")
    a = A.Graph.from_problem(p)
    assert a.info()["driver"] == A.DRIVER_RESIDENT      # chosen automatically
    a.run(37)
    b = A.Graph.from_problem(p)
    b.run(20)
    b.run(17)
    assert np.array_equal(a.z(), b.z()) and np.array_equal(a.u(), b.u())
    assert np.array_equal(a.x(), b.x())
    c = A.Graph.from_problem(p)
    xm, zm = c.run_profiled(37)
    assert xm > 0 and zm == 0
    assert np.array_equal(a.z(), c.z())
    # the state set from the host is what the next resident run starts from
    d = A.Graph.from_problem(p)
    d.set_state(a.z(), a.u())
    d.run(5)
    a.run(5)
    assert np.array_equal(a.z(), d.z())


def _split_centres_radii(p):
    """The same packing with variables reordered as all centres, then all
    radii: pair-tile entities then need their z offsets from the table."""
    N = p.var_dims.size // 2
    new = np.empty(2 * N, dtype=np.int64)
    new[0::2] = np.arange(N)
    new[1::2] = N + np.arange(N)
    dims = np.r_[np.full(N, 2, np.int32), np.ones(N, np.int32)]
    z_old = p.z0.reshape(N, 3)
    z0 = np.r_[z_old[:, :2].ravel(), z_old[:, 2]]
    groups = [W.FactorGroup(gr.kind, new[gr.var_ids].astype(np.int32), gr.params, gr.shared)
              for gr in p.groups]
    return W.Problem(p.name + "_split", dims, groups, z0, rho=p.rho, alpha=p.alpha)


@pytest.mark.parametrize("pair_state", [A.PAIR_STATE_AUTO, A.PAIR_STATE_DENSE])
def test_pair_tiles_with_entity_table(pair_state):
    p = _split_centres_radii(W.packing(130, "square", 0.3 / np.sqrt(130), seed=7))
    g = A.Graph.from_problem(p, driver=A.DRIVER_LAUNCHES, pair_state=pair_state)
    assert g.info()["n_pair_tiles"] > 0
    _one_step(p, 30, FP32, 1e-5, steps=3, driver=A.DRIVER_LAUNCHES, pair_state=pair_state)
    _traj(p, 12, FP64, 1e-9, driver=A.DRIVER_LAUNCHES)


@pytest.mark.parametrize("pair_state", [A.PAIR_STATE_AUTO, A.PAIR_STATE_DENSE])
def test_full_size_packing_5000_steps(pair_state):
    """5000 disks (3160 tiles, state beyond the Infinity Cache): three steps
    from a common state against the oracle, both pair states."""
    _one_step(W.workload("packing_sq5000"), 10, FP32, 1e-5, steps=3, pair_state=pair_state)


def _multiplicity_graph(counts, seed):
    """Scalar variables, variable i carrying counts[i] quadratic factors
    (weights U[0.1, 2]): z-lists of every class and stride layout (long
    lists, medium lists of mixed length, short lists, an empty list)."""
    rng = np.random.default_rng(seed)
    ids = np.repeat(np.arange(len(counts), dtype=np.int32), counts)
    groups = [W.FactorGroup("quad", ids[:, None], rng.uniform(0.1, 2.0, (ids.size, 1)))]
    z0 = rng.standard_normal(len(counts))
    return W.Problem("multiplicity", np.ones(len(counts), np.int32), groups, z0)


@pytest.mark.parametrize("driver", [A.DRIVER_LAUNCHES, A.DRIVER_RESIDENT])
def test_zlist_classes_and_layouts(driver):
    # one list of 200 (one workgroup), one of 100 and 1000 of 5 (medium lists
    # too uneven to pad: explicit ranges), 40 of 3 (short), one of 0
    counts = np.r_[200, 100, np.full(1000, 5), np.full(40, 3), 0]
    p = _multiplicity_graph(counts, seed=17)
    if driver == A.DRIVER_RESIDENT:     # small enough for the LDS image in FP64
        p = _multiplicity_graph(np.r_[150, 60, np.full(150, 5), np.full(20, 3), 0], seed=18)
    g, o = _traj(p, 30, FP64, 1e-9, driver=driver)
    assert g.info()["driver"] == driver
    assert g.z()[-1] == p.z0[-1]
    _traj(p, 30, FP32, 1e-4, driver=driver)
    # medium lists of equal length: padded stride layout
    nq = 500 if driver == A.DRIVER_LAUNCHES else 100
    q = _multiplicity_graph(np.r_[np.full(nq, 7), np.full(10, 2)], seed=19)
    _traj(q, 30, FP64, 1e-9, driver=driver)
