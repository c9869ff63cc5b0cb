"""The oracle's OpenMP build (the paper's first CPU scheme: each update a
parallel loop over its own index) computes every element with the same
arithmetic in the same order as the serial build, so the two agree bit for
bit on every graph family, including the stopping iteration."""
import numpy as np
import pytest

import oracle as O
import workloads as W


def _cases():
    inst = W.mpc_batch(1, seed=45)[0]
    return {
        "packing_40": W.packing(40, "square", 0.1, seed=5),
        "svm_300_d4": W.svm(300, 4, seed=6),
        "svm_copies_25_d3": W.svm_copies(25, 3, seed=7),
        "mpc": W.mpc_graph(inst),
    }


@pytest.mark.parametrize("name", ["packing_40", "svm_300_d4", "svm_copies_25_d3", "mpc"])
def test_openmp_build_is_bitwise_serial(name):
    p = _cases()[name]
    a = O.OracleGraph(p)
    b = O.OracleGraph(p, openmp=True)
    assert b._L.orc_threads() >= 1
    a.run(40)
    b.run(40)
    assert np.array_equal(a.z, b.z) and np.array_equal(a.u, b.u) and np.array_equal(a.x, b.x)
    assert a.residuals() == b.residuals()
    ka = a.run(5000, tol=1e-6)
    kb = b.run(5000, tol=1e-6)
    assert ka == kb and np.array_equal(a.z, b.z)


@pytest.mark.parametrize("name", ["packing_40", "svm_300_d4", "svm_copies_25_d3", "mpc"])
def test_one_region_scheme_is_bitwise_serial(name):
    """The paper's second CPU scheme (one parallel region for the whole run,
    barriers between update types) also computes the serial iteration bit
    for bit, stopping iteration included, in both builds."""
    p = _cases()[name]
    a = O.OracleGraph(p)
    b = O.OracleGraph(p, openmp=True)
    c = O.OracleGraph(p)
    a.run(40)
    b.run(40, region=True)
    c.run(40, region=True)
    for g in (b, c):
        assert np.array_equal(a.z, g.z) and np.array_equal(a.u, g.u) and np.array_equal(a.x, g.x)
        assert a.residuals() == g.residuals()
    ka = a.run(5000, tol=1e-6)
    kb = b.run(5000, tol=1e-6, region=True)
    assert ka == kb and np.array_equal(a.z, b.z) and a.residuals() == b.residuals()
