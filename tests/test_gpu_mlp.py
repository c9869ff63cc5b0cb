"""GPU MLP (matrix-core bf16 products, fp32 accumulation) against the FP64
oracle MLP run on the same weights with the same bf16 operand rounding."""
import numpy as np
import pytest

from oracle import warmstart as WS
from tests.helpers import rel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _net(n_in, hid, n_out, batch, seed):
    from paper_1603_02526_amd import mlp as MLPm
    net = MLPm.MLP(n_in, hid, n_out, max_batch=batch)
    flat = MLPm.init_params(n_in, hid, n_out, seed)
    flat[-n_out:] = np.random.default_rng(seed + 1).standard_normal(n_out) * 0.1
    net.set_params(flat)
    return net, flat


@pytest.mark.parametrize("n_in,hid,n_out,batch", [(8, 256, 1100, 300), (5, 64, 37, 77),
                                                  (12, 128, 200, 1024)])
def test_forward_matches_oracle(n_in, hid, n_out, batch):
    net, flat = _net(n_in, hid, n_out, batch, 11)
    x = np.random.default_rng(2).standard_normal((batch, n_in)).astype(np.float32)
    y = torch.zeros((batch, n_out), device="cuda")
    net.forward(torch.tensor(x, device="cuda"), y)
    torch.cuda.synchronize()
    params = WS.unflatten(flat, n_in, hid, n_out)
    yo, _ = WS.mlp_forward(params, x.astype(np.float64), bf16=True)
    assert rel(y.cpu().numpy(), yo) < 1e-3, rel(y.cpu().numpy(), yo)
    # and the bf16 network is close to the exact one
    ye, _ = WS.mlp_forward(params, x.astype(np.float64), bf16=False)
    assert rel(yo, ye) < 3e-2


@pytest.mark.parametrize("n_in,hid,n_out,batch", [(8, 256, 1100, 256), (6, 64, 50, 130)])
def test_gradients_match_oracle(n_in, hid, n_out, batch):
    net, flat = _net(n_in, hid, n_out, batch, 21)
    rng = np.random.default_rng(3)
    x = rng.standard_normal((batch, n_in)).astype(np.float32)
    tg = rng.standard_normal((batch, n_out)).astype(np.float32)
    g = torch.zeros(net.n_params, device="cuda")
    loss = torch.zeros(1, device="cuda")
    net.grads(torch.tensor(x, device="cuda"), torch.tensor(tg, device="cuda"), g, loss)
    torch.cuda.synchronize()
    params = WS.unflatten(flat, n_in, hid, n_out)
    lo, go = WS.mlp_loss_grad(params, x.astype(np.float64), tg.astype(np.float64), bf16=True)
    assert abs(loss.item() - lo) < 1e-4 * abs(lo)
    gg = WS.unflatten(g.cpu().numpy(), n_in, hid, n_out)
    for a, b in zip(gg, go):
        assert rel(a, b) < 1e-3, rel(a, b)


def test_adam_step_matches_oracle_and_training_lowers_loss():
    n_in, hid, n_out, batch = 6, 64, 40, 512
    net, flat = _net(n_in, hid, n_out, batch, 31)
    rng = np.random.default_rng(4)
    x = rng.standard_normal((batch, n_in)).astype(np.float32)
    Wt = rng.standard_normal((n_out, n_in))
    tg = (np.tanh(x @ Wt.T)).astype(np.float32)
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(tg, device="cuda")
    # one step against the oracle's Adam on the oracle's gradient
    net.train_step(xd, td, 1e-3)
    torch.cuda.synchronize()
    params = WS.unflatten(flat, n_in, hid, n_out)
    _, go = WS.mlp_loss_grad(params, x.astype(np.float64), tg.astype(np.float64), bf16=True)
    m = [np.zeros_like(p) for p in params]
    v = [np.zeros_like(p) for p in params]
    WS.adam_step(params, go, m, v, 1, 1e-3)
    after = net.get_params().astype(np.float64)
    assert rel(after, WS.flatten(params)) < 1e-4
    loss = torch.zeros(1, device="cuda")
    net.grads(xd, td, None, loss)
    l0 = loss.item()
    for _ in range(300):
        net.train_step(xd, td, 3e-3)
    net.grads(xd, td, None, loss)
    torch.cuda.synchronize()
    assert loss.item() < 0.3 * l0


def test_output_scaling_forward_and_gradients():
    """With a fixed output affine y = mean + sd * yhat the forward output is
    denormalised and the loss is taken on (target - mean) / sd."""
    n_in, hid, n_out, batch = 8, 64, 90, 200
    net, flat = _net(n_in, hid, n_out, batch, 41)
    rng = np.random.default_rng(8)
    mean = rng.standard_normal(n_out).astype(np.float32) * 0.3
    sd = (0.05 + rng.random(n_out)).astype(np.float32)
    x = rng.standard_normal((batch, n_in)).astype(np.float32)
    tg = (mean + sd * rng.standard_normal((batch, n_out))).astype(np.float32)
    net.set_output_scaling(mean, sd)
    xd, td = torch.tensor(x, device="cuda"), torch.tensor(tg, device="cuda")
    y = torch.zeros((batch, n_out), device="cuda")
    net.forward(xd, y)
    g = torch.zeros(net.n_params, device="cuda")
    loss = torch.zeros(1, device="cuda")
    net.grads(xd, td, g, loss)
    torch.cuda.synchronize()
    params = WS.unflatten(flat, n_in, hid, n_out)
    yo, _ = WS.mlp_forward(params, x.astype(np.float64), bf16=True, mean=mean, sd=sd)
    assert rel(y.cpu().numpy(), yo) < 1e-3
    lo, go = WS.mlp_loss_grad(params, x.astype(np.float64), tg.astype(np.float64), bf16=True,
                              mean=mean.astype(np.float64), sd=sd.astype(np.float64))
    assert abs(loss.item() - lo) < 1e-4 * abs(lo)
    for a, b in zip(WS.unflatten(g.cpu().numpy(), n_in, hid, n_out), go):
        assert rel(a, b) < 1e-3
    # fitting the affine from data gives the columns' mean and spread
    net.fit_output_scaling(td, sd_min=1e-6)
    m2, s2 = net.get_output_scaling()
    np.testing.assert_allclose(m2, tg.astype(np.float64).mean(0), rtol=1e-4, atol=1e-6)
    np.testing.assert_allclose(s2, tg.astype(np.float64).std(0), rtol=1e-4)
