"""Pins of the oracle's helper computations against definitions that do not
come from the oracle itself.

* ``adam_step`` against torch's Adam (Kingma & Ba, bias-corrected) in FP64;
* ``mlp_forward`` against torch's linear and ReLU layers in FP64, without
  and with bf16 operand rounding (torch's own float32 -> bfloat16 cast
  applied to both operands of every product), and ``mlp_loss_grad``
  against torch autograd;
* the residuals r = max_e |x_e - z_b| and s = rho max_b |z_b - z_b^prev|
  (the stopping measures used throughout, Sec. II leaves them open)
  recomputed in numpy from the iterates around one step;
* ``packing_objective``, ``svm_objective`` and ``mpc_objective`` on small
  cases worked out by hand (Sec. V problem definitions).
"""
import dataclasses
import types

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import warmstart as WS


def _rand_params(rng, n_in, hidden, n_out, scale=0.5):
    return [rng.standard_normal(s) * scale for s in WS.mlp_shapes(n_in, hidden, n_out)]


def test_adam_step_matches_torch_adam():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(11)
    params = _rand_params(rng, 4, 6, 3)
    tp = [torch.nn.Parameter(torch.tensor(p.copy(), dtype=torch.float64)) for p in params]
    opt = torch.optim.Adam(tp, lr=3e-2, betas=(0.9, 0.999), eps=1e-8)
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    for step in range(1, 4):
        grads = [rng.standard_normal(p.shape) for p in params]
        WS.adam_step(params, grads, m, v, step, 3e-2)
        for t, g in zip(tp, grads):
            t.grad = torch.tensor(g, dtype=torch.float64)
        opt.step()
        for p, t in zip(params, tp):
            np.testing.assert_allclose(p, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def _torch_mlp(torch, params, x, bf16, mean=None, sd=None):
    F = torch.nn.functional
    W1, b1, W2, b2, W3, b3 = [torch.tensor(p, dtype=torch.float64) for p in params]
    X = torch.tensor(x, dtype=torch.float64)

    def rnd(a):
        return a.to(torch.float32).to(torch.bfloat16).to(torch.float64) if bf16 else a

    h1 = F.relu(F.linear(rnd(X), rnd(W1), b1))
    h2 = F.relu(F.linear(rnd(h1), rnd(W2), b2))
    y = F.linear(rnd(h2), rnd(W3), b3)
    if mean is not None:
        y = torch.tensor(mean) + torch.tensor(sd) * y
    return y


@pytest.mark.parametrize("bf16", [False, True])
def test_mlp_forward_matches_torch_layers(bf16):
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(12)
    params = _rand_params(rng, 8, 16, 5)
    x = rng.standard_normal((9, 8))
    mean, sd = rng.standard_normal(5), rng.uniform(0.5, 2.0, 5)
    y, _ = WS.mlp_forward(params, x, bf16)
    ref = _torch_mlp(torch, params, x, bf16).numpy()
    np.testing.assert_allclose(y, ref, rtol=1e-12, atol=1e-12)
    # the output affine y = mean + sd * yhat
    y2, _ = WS.mlp_forward(params, x, bf16, mean=mean, sd=sd)
    np.testing.assert_allclose(y2, _torch_mlp(torch, params, x, bf16, mean, sd).numpy(),
                               rtol=1e-12, atol=1e-12)
    # a plausible mistake (ReLU on the output) would differ: outputs are negative somewhere
    assert (ref < 0).any()


def test_mlp_loss_grad_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(13)
    params = _rand_params(rng, 4, 7, 3)
    x = rng.standard_normal((6, 4))
    t = rng.standard_normal((6, 3))
    mean, sd = rng.standard_normal(3), rng.uniform(0.5, 2.0, 3)
    loss, grads = WS.mlp_loss_grad(params, x, t, mean=mean, sd=sd)
    tp = [torch.tensor(p, dtype=torch.float64, requires_grad=True) for p in params]
    F = torch.nn.functional
    X = torch.tensor(x)
    yhat = F.linear(F.relu(F.linear(F.relu(F.linear(X, tp[0], tp[1])), tp[2], tp[3])), tp[4], tp[5])
    tl = F.mse_loss(yhat, torch.tensor((t - mean) / sd), reduction="mean")
    tl.backward()
    assert abs(loss - tl.item()) <= 1e-12 * abs(tl.item())
    for g, p in zip(grads, tp):
        np.testing.assert_allclose(g, p.grad.numpy(), rtol=1e-11, atol=1e-13)


def _weighted(p, weights):
    groups = [dataclasses.replace(g, rho=weights.get(i)) for i, g in enumerate(p.groups)]
    return dataclasses.replace(p, groups=groups)


def _var_rho(p):
    """Per z scalar, the largest rho of the edges that reach it."""
    off = p.var_offsets()
    out = np.zeros(p.n_scalars)
    for g in p.groups:
        r = p.rho if g.rho is None else g.rho
        for vid in np.unique(g.var_ids):
            sl = slice(off[vid], off[vid] + p.var_dims[vid])
            out[sl] = np.maximum(out[sl], r)
    return out


@pytest.mark.parametrize("case", ["packing", "svm", "packing_weighted", "mpc"])
def test_residuals_recomputed_from_iterates(case):
    if case == "packing":
        p = W.packing(7, "triangle", 0.1, seed=61)
    elif case == "svm":
        p = W.svm(30, 4, seed=62)
    elif case == "packing_weighted":
        p = _weighted(W.packing(7, "square", 0.15, seed=63), {0: 2.0, 2: 3.0})
    else:
        p = W.mpc_graph(W.mpc_batch(1, seed=64, T_range=(10, 14))[0])
    g = O.OracleGraph(p)
    sz = g.slot_z
    vr = _var_rho(p)
    for k in (1, 5, 17):
        g.run(k)
        zprev = g.z
        g.run(1)
        x, z = g.x, g.z
        r, s = g.residuals()
        assert r == np.max(np.abs(x - z[sz]))
        assert s == np.max(vr * np.abs(z - zprev))
        assert r > 0.0 and s > 0.0


def _fake_packing(z, walls, gamma=0.5):
    return types.SimpleNamespace(meta=dict(gamma=gamma, walls=walls))


def test_packing_objective_hand_cases():
    floor = [((0.0, 1.0), (0.0, 0.0))]  # y >= r
    # disk 1 at (0.2, 0.04), r 0.1: 0.06 below the floor's allowance;
    # disk 2 at (0.35, 0.3), r 0.05: distance 0.300167 > 0.15, no overlap
    z = np.array([0.2, 0.04, 0.1, 0.35, 0.3, 0.05])
    o = O.packing_objective(_fake_packing(z, floor), z)
    assert o["objective"] == pytest.approx(-0.25 * (0.01 + 0.0025), rel=1e-14)
    assert o["area"] == pytest.approx(np.pi * 0.0125, rel=1e-14)
    assert o["max_violation"] == pytest.approx(0.06, rel=1e-12)
    # overlapping pair, 0.3 apart with radii 0.2 and 0.25: violation 0.15
    z = np.array([0.5, 0.5, 0.2, 0.8, 0.5, 0.25])
    o = O.packing_objective(_fake_packing(z, floor), z)
    assert o["max_violation"] == pytest.approx(0.15, rel=1e-12)
    # feasible: touching disks inside the floor's half-plane
    z = np.array([0.5, 0.5, 0.1, 0.7, 0.5, 0.1])
    o = O.packing_objective(_fake_packing(z, floor), z)
    assert o["max_violation"] == pytest.approx(0.0, abs=1e-15)
    # a negative radius counts as its own violation
    z = np.array([0.5, 0.5, -0.07, 0.9, 0.9, 0.01])
    o = O.packing_objective(_fake_packing(z, floor, gamma=2.0), z)
    assert o["max_violation"] == pytest.approx(0.07, rel=1e-12)
    assert o["objective"] == pytest.approx(-(0.0049 + 0.0001), rel=1e-12)
    # the paper's triangle: the incircle (r = sqrt(3)/6) touches all three walls
    p = W.packing(1, "triangle", 0.1, seed=1)
    zi = np.array([0.5, np.sqrt(3) / 6, np.sqrt(3) / 6])
    assert O.packing_objective(p, zi)["max_violation"] < 1e-15
    zi[2] += 1e-3
    assert O.packing_objective(p, zi)["max_violation"] == pytest.approx(1e-3, rel=1e-9)


def test_svm_objective_hand_case():
    # d = 1, w = 2, b = -1, points a = (1, 0, 2) with y = (+1, -1, +1):
    # margins y(wa+b) = 1, 1, 3 -> hinge 0, 0, 0; then b = 0: 2, 0, 4 -> hinge 0, 1, 0
    prob = types.SimpleNamespace(meta=dict(d=1, a=np.array([[1.0], [0.0], [2.0]]),
                                           y=np.array([1.0, -1.0, 1.0]), C=3.0, l2_weight=1.0))
    assert O.svm_objective(prob, np.array([2.0, -1.0])) == pytest.approx(2.0, rel=1e-15)
    assert O.svm_objective(prob, np.array([2.0, 0.0])) == pytest.approx(2.0 + 3.0, rel=1e-15)


def test_mpc_objective_hand_case():
    # T = 2, n = 1, m = 1: x1 = a x0 + b u0, x2 = a x1 + b u1
    inst = types.SimpleNamespace(T=2, n=1, m=1, A=np.array([[0.5]]), B=np.array([[2.0]]),
                                 q=np.array([1.0]), r=np.array([0.1]), u_box=1.0,
                                 x0=np.array([1.0]))
    # u0 = 0.25 -> x1 = 1.0; u1 = -1.5 -> x2 = -2.5 (box violated by 0.5)
    z = np.array([0.25, 1.0, -1.5, -2.5])
    o = O.mpc_objective(inst, z)
    assert o["cost"] == pytest.approx(0.5 * (1.0 + 6.25) + 0.05 * (0.0625 + 2.25), rel=1e-15)
    assert o["dyn_violation"] == pytest.approx(0.0, abs=1e-15)
    assert o["box_violation"] == pytest.approx(0.5, rel=1e-15)
    z[3] = -2.0
    assert O.mpc_objective(inst, z)["dyn_violation"] == pytest.approx(0.5, rel=1e-15)
