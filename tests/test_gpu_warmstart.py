"""Learned warm start end to end on a small system: data from the GPU
solver, training with the GPU kernels, then warm solves (network + dual
completion) against cold solves on fresh initial states."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def test_trained_warm_start_beats_cold_start():
    from paper_1603_02526_amd import warmstart as WSm
    rng = np.random.default_rng(5)
    A, B = W.mpc_system(rng, 4, 2)
    sys_ = WSm.System(A, B, 30, np.ones(4), np.full(2, 0.1), 1.0)
    ws = WSm.WarmStart(sys_, batch=1024, hidden=128, init_seed=1)
    X, Z = ws.generate(65536, seed=11)
    hist = ws.train(X, Z, epochs=20, lr=1e-3, lr_final=1e-4)
    assert hist[-1] < 0.2 * hist[0]
    x0 = torch.tensor(np.random.default_rng(12).standard_normal((1024, 4)).astype(np.float32),
                      device="cuda")
    zc, itc = ws.solve(x0, "cold")
    torch.cuda.synchronize()
    zc, itc = zc.cpu().numpy().copy(), ws.iters.cpu().numpy().copy()
    zw, _ = ws.solve(x0, "warm")
    torch.cuda.synchronize()
    zw, itw = zw.cpu().numpy().copy(), ws.iters.cpu().numpy().copy()
    assert np.all(itc > 0) and np.all(itw > 0)          # both meet the residual
    assert itw.mean() < 0.8 * itc.mean(), (itw.mean(), itc.mean())
    # z alone (no dual completion) is no better than a cold start
    ws.solve(x0, "warm_z")
    torch.cuda.synchronize()
    itz = ws.iters.cpu().numpy().copy()
    assert itz.mean() > 0.9 * itc.mean(), (itz.mean(), itc.mean())
    # both are solutions to the same tolerance: trajectories agree closely
    err = np.abs(zw - zc).max()
    assert err < 5e-3, err
