"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/admm.h, validates graphs and reports layout sizes.
No compute call is made here."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_1603_02526_amd import admm as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            txt = open(os.path.join(inc, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(admm_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    L = A.lib()
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(L, n), n
    assert L.admm_abi_version() == 1


def _finalize_cpu(g):
    """finalize on a machine without a GPU validates and reports NO_DEVICE."""
    try:
        g.finalize(0)
        return A.OK
    except A.AdmmError as e:
        return e.status


def _expected_tiles(N, rb):
    """Tiles of rb x 64 disks holding at least one pair i < j (brute force)."""
    return len({(i // rb, j // 64) for i in range(N) for j in range(i + 1, N)})


@pytest.mark.parametrize("name,N", [("packing_tri10", 10), ("packing_sq2000", 2000)])
@pytest.mark.parametrize("rb", [16, 32, 64])
def test_packing_layout(name, N, rb):
    p = W.workload(name)
    g = A.Graph.from_problem(p, device=None, pair_rows=rb, driver=A.DRIVER_LAUNCHES)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    inf = g.info()
    assert inf["n_edges"] == p.n_edges and inf["n_slots"] == p.n_slots
    assert inf["n_factors"] == p.n_factors and inf["n_scalars"] == p.n_scalars
    assert inf["n_buckets"] == 3
    assert inf["n_pair_tiles"] == _expected_tiles(N, rb)
    # algorithmic bytes: m read + write per slot, plus wall/radius/pair data
    assert inf["algo_bytes_per_iter"] >= 8 * p.n_slots


def test_driver_selection():
    # small graphs: resident in LDS, no pair tiles; forced launches keep tiles
    p = W.workload("packing_tri10")
    g = A.Graph.from_problem(p, device=None)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    inf = g.info()
    assert inf["driver"] == A.DRIVER_RESIDENT and inf["n_pair_tiles"] == 0
    # the image holds at least the pool (contributions, m and x) and two z copies
    assert inf["resident_lds_bytes"] >= 4 * (inf["n_contributions"] + 2 * p.n_slots + 2 * p.n_scalars)
    assert inf["resident_lds_bytes"] <= 96 * 1024
    g = A.Graph.from_problem(p, device=None, driver=A.DRIVER_LAUNCHES)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    inf = g.info()
    assert inf["driver"] == A.DRIVER_LAUNCHES and inf["n_pair_tiles"] == 1
    assert inf["resident_lds_bytes"] == 0
    # large graphs: recorded iteration blocks (or launches when asked for);
    # the resident driver is refused
    p = W.workload("packing_sq2000")
    g = A.Graph.from_problem(p, device=None)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    assert g.info()["driver"] == A.DRIVER_GRAPH
    g = A.Graph.from_problem(p, device=None, driver=A.DRIVER_LAUNCHES)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    assert g.info()["driver"] == A.DRIVER_LAUNCHES
    g = A.Graph.from_problem(p, device=None, driver=A.DRIVER_GRAPH, graph_block=8)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    assert g.info()["driver"] == A.DRIVER_GRAPH
    for bad in (1, 3, 5000, -2):
        with pytest.raises(A.AdmmError) as e:
            A.Graph.from_problem(p, device=None, graph_block=bad)
        assert e.value.status == A.E_ARG
    g = A.Graph.from_problem(p, device=None, driver=A.DRIVER_RESIDENT)
    assert _finalize_cpu(g) == A.E_UNSUPPORTED
    # FP64 doubles the image: a graph that fits in FP32 may not in FP64
    q = W.svm(1500, 4, seed=5)
    g32 = A.Graph.from_problem(q, device=None)
    g64 = A.Graph.from_problem(q, precision=A.FP64, device=None)
    assert _finalize_cpu(g32) in (A.OK, A.E_NO_DEVICE)
    assert _finalize_cpu(g64) in (A.OK, A.E_NO_DEVICE)
    i32, i64 = g32.info(), g64.info()
    if i64["driver"] == A.DRIVER_RESIDENT:
        assert i64["resident_lds_bytes"] > i32["resident_lds_bytes"]


def test_sparse_pair_state_selection():
    p = W.workload("packing_sq2000")
    for kw, want in ((dict(), 1), (dict(pair_state=A.PAIR_STATE_DENSE), 0),
                     (dict(precision=A.FP64), 0), (dict(alpha=1.5), 0)):
        g = A.Graph.from_problem(p, device=None, **kw)
        assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
        assert g.info()["sparse_pair_state"] == want, kw


def test_svm_layout():
    p = W.svm(5000, 20, seed=3)
    g = A.Graph.from_problem(p, device=None)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    inf = g.info()
    assert inf["n_edges"] == 5000 * 21 + 20
    assert inf["n_pair_tiles"] == 0
    # one partial per variable per 256-factor workgroup (FP32: four lanes
    # per four factors for d <= 32), plus 20 L2 slots
    assert inf["n_contributions"] == 20 * 21 + 20
    # FP64: two lanes per factor, 128 factors per workgroup
    g = A.Graph.from_problem(p, device=None, precision=A.FP64)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    assert g.info()["n_contributions"] == 40 * 21 + 20


def test_copies_svm_layout():
    N, d = 3000, 20
    p = W.svm_copies(N, d, seed=4)
    g = A.Graph.from_problem(p, device=None)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    inf = g.info()
    assert inf["n_edges"] == p.n_edges and inf["n_slots"] == p.n_slots
    # margin, minimal-error, norm and equality buckets
    assert inf["n_buckets"] == 4
    # every slot contributes its m directly, except the shared bias: one
    # partial per 256-factor workgroup of the margin bucket
    assert inf["n_contributions"] == p.n_slots - N + (N + 255) // 256


def test_group_rho_state_and_radius_check():
    g = A.Graph([2, 1])
    g.add_factors("radius", [[1]], [0.5], shared=True)
    g.set_group_rho(0, 0.4)                     # the group's rho must exceed gamma
    _expect(A.E_NUMERIC, g.finalize, 0)
    g = A.Graph([2, 1])
    g.add_factors("radius", [[1]], [0.5], shared=True)
    g.set_group_rho(0, 0.9)
    g.set_rho(0.3)                              # the graph's rho no longer applies to it
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    g = A.Graph([1])
    g.add_factors("quad", [[0]], [2.0], True)
    _expect(A.E_ARG, g.set_group_alpha, 0, -1.0)
    _expect(A.E_ARG, g.set_group_alpha, 3, 1.5)
    # a group alpha other than 1 switches the whole graph to the (m, x) state
    p = W.packing(5, "square", 0.1, seed=9)
    p.groups[2] = W.FactorGroup(p.groups[2].kind, p.groups[2].var_ids, p.groups[2].params,
                                p.groups[2].shared, alpha=1.5)
    g = A.Graph.from_problem(p, device=None)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    assert g.info()["alpha_is_one"] == 0


def test_incomplete_pairs_fall_back_to_general_layout():
    p = W.packing(12, "square", 0.05, seed=2)
    g0 = p.groups[0]
    p.groups[0] = W.FactorGroup("nonoverlap", g0.var_ids[:-1], g0.params, True)
    g = A.Graph.from_problem(p, device=None)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    assert g.info()["n_pair_tiles"] == 0


def _expect(status, fn, *args):
    with pytest.raises(A.AdmmError) as ei:
        fn(*args)
    assert ei.value.status == status, str(ei.value)


def test_validation_errors():
    g = A.Graph([2, 1, 2, 1])
    _expect(A.E_ARG, g.add_factors, "nonoverlap", [[0, 1, 2, 7]])        # bad id
    _expect(A.E_ARG, g.add_factors, "nonoverlap", [[0, 1, 2, 2]])        # repeated
    _expect(A.E_ARG, g.add_factors, "wall", [[0, 1]], [[1.0, 0.0]])      # param_len
    _expect(A.E_ARG, g.add_factors, "nonoverlap", [[0, 1, 3, 2]])        # wrong dims
    g = A.Graph([2, 1])
    g.add_factors("radius", [[1]], [1.0], shared=True)
    _expect(A.E_NUMERIC, g.finalize, 0)                                   # rho <= gamma
    g = A.Graph([1, 1, 1])
    _expect(A.E_ARG, g.add_factors, "hinge", [[0, 1, 2]], [[1.0, 2.0, 1.0, -1.0]])  # C < 0
    g = A.Graph([3])
    _expect(A.E_ARG, g.add_factors, "quad", [[0]], [[1.0, 2.0]])          # weight short
    g = A.Graph([3])
    _expect(A.E_ARG, g.add_factors, "box", [[0]], [1.0, -1.0], True)     # lo > hi
    g = A.Graph([2, 1, 1])
    _expect(A.E_ARG, g.add_factors, "margin", [[0, 1, 2]], [[1.0, 2.0, 0.5]])   # y not +-1
    _expect(A.E_ARG, g.add_factors, "margin", [[0, 1, 2]], [[1.0, 1.0]])        # param_len
    _expect(A.E_ARG, g.add_factors, "margin", [[1, 0, 2]], [[1.0, 1.0]])        # dims (1,2,1)
    _expect(A.E_ARG, g.add_factors, "equal", [[0, 1]])                          # dims 2 vs 1
    _expect(A.E_ARG, g.add_factors, "minerr", [[1]], [-1.0], True)              # lambda < 0
    g = A.Graph([1, 1])
    g.add_factors("quad", [[0], [1]], [2.0], True)
    _expect(A.E_ARG, g.set_group_rho, 1, 2.0)                             # no group 1
    _expect(A.E_ARG, g.set_group_rho, 0, 0.0)                             # rho <= 0
    _expect(A.E_ARG, g.set_group_rho, -1, 2.0)
    g.set_group_rho(0, 2.0)
    _expect(A.E_ARG, A.Graph, [1, 0])                                      # dim 0
    _expect(A.E_ARG, A.Graph, [1], 7)                                      # precision
    g = A.Graph([1])
    _expect(A.E_ARG, g.set_rho, -1.0)
    _expect(A.E_ARG, g.set_alpha, 0.0)
    _expect(A.E_ARG, g.set_option, A.OPT_PAIR_ROWS, 48)
    _expect(A.E_ARG, g.set_option, A.OPT_DRIVER, 4)
    _expect(A.E_ARG, g.set_option, A.OPT_GRAPH_BLOCK, 7)
    _expect(A.E_ARG, g.set_option, A.OPT_PAIR_STATE, 2)
    _expect(A.E_ARG, g.set_option, 99, 1)


def test_state_machine():
    g = A.Graph([1])
    g.add_factors("l2", [[0]], [1.0], shared=True)
    _expect(A.E_STATE, g.run, 1)
    _expect(A.E_STATE, g.z)
    st = _finalize_cpu(g)
    if st == A.E_NO_DEVICE:
        _expect(A.E_STATE, g.run, 1)
        _expect(A.E_STATE, g.add_factors, "l2", [[0]], [1.0], True)
        _expect(A.E_STATE, g.set_rho, 2.0)


def test_lindyn_limits_and_shapes():
    inst = W.mpc_batch(1, seed=9)[0]
    p = W.mpc_graph(inst)
    g = A.Graph.from_problem(p, device=None)
    assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
    assert g.info()["n_slots"] == p.n_slots == inst.T * (3 * inst.n + 3 * inst.m) - inst.n
    # n above the register-resident limit is refused, not silently slowed
    rng = np.random.default_rng(0)
    A_, B_ = W.mpc_system(rng, 20, 2)
    big = W.MPCInstance(5, 20, 2, A_, B_, np.zeros(20), np.ones(20), np.ones(2), 1.0)
    g = A.Graph.from_problem(W.mpc_graph(big), device=None)
    _expect(A.E_UNSUPPORTED, g.finalize, 0)


def test_mpc_batch_validation_before_device():
    from paper_1603_02526_amd import mpc as M
    rng = np.random.default_rng(1)
    A_, B_ = W.mpc_system(rng, 13, 2)
    bad = W.MPCInstance(10, 13, 2, A_, B_, np.zeros(13), np.ones(13), np.ones(2), 1.0)
    _expect(A.E_UNSUPPORTED, M.MPCBatch, [bad])
    A_, B_ = W.mpc_system(rng, 4, 5)
    bad = W.MPCInstance(10, 4, 5, A_, B_, np.zeros(4), np.ones(4), np.ones(5), 1.0)
    _expect(A.E_UNSUPPORTED, M.MPCBatch, [bad])
    A_, B_ = W.mpc_system(rng, 4, 2)
    bad = W.MPCInstance(257, 4, 2, A_, B_, np.zeros(4), np.ones(4), np.ones(2), 1.0)
    _expect(A.E_UNSUPPORTED, M.MPCBatch, [bad])
    neg = W.MPCInstance(10, 4, 2, A_, B_, np.zeros(4), -np.ones(4), np.ones(2), 1.0)
    _expect(A.E_ARG, M.MPCBatch, [neg])
    ok = W.MPCInstance(10, 4, 2, A_, B_, np.zeros(4), np.ones(4), np.ones(2), 1.0)
    _expect(A.E_ARG, M.MPCBatch, [ok], -1.0)


def test_three_weight_validation():
    """The three-weight variant is validated before any device call: packing
    graphs pass (pair tiles with the sparse state in FP32, the general layout
    in FP64 or with the dense pair state), other graphs, alpha != 1 and the
    resident driver are refused."""
    p = W.workload("packing_tri10")
    for prec, dense, tiles in ((A.FP32, False, True), (A.FP64, False, False), (A.FP32, True, False)):
        g = A.Graph.from_problem(p, precision=prec, device=None, three_weight=True,
                                 pair_state=A.PAIR_STATE_DENSE if dense else A.PAIR_STATE_AUTO)
        assert _finalize_cpu(g) in (A.OK, A.E_NO_DEVICE)
        inf = g.info()
        assert inf["three_weight"] == 1 and (inf["n_pair_tiles"] > 0) == tiles
        assert inf["driver"] == A.DRIVER_GRAPH
    for q, kw in ((W.svm(300, 3, seed=1), {}), (p, dict(alpha=1.5)),
                  (p, dict(driver=A.DRIVER_RESIDENT))):
        g = A.Graph.from_problem(q, device=None, three_weight=True, **kw)
        assert _finalize_cpu(g) == A.E_UNSUPPORTED
    _expect(A.E_ARG, A.Graph([1]).set_option, A.OPT_THREE_WEIGHT, 2)
