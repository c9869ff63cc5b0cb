"""The allocation-free output-scaling fit (admm_mlp_fit_output_scaling_noalloc)
against the allocating one, through the C ABI: identical means and spreads
on two calls in a row (the second on a smaller input), and sizes beyond the
fixed workspace refused."""
import numpy as np
import pytest

from paper_1603_02526_amd import admm as A
from paper_1603_02526_amd import mlp as MLPm

pytestmark = pytest.mark.gpu


def _fit(net, y, noalloc):
    import torch
    if noalloc:
        net.fit_output_scaling_noalloc(y, sd_min=1e-4, stream=torch.cuda.current_stream())
    else:
        net.fit_output_scaling(y, sd_min=1e-4, stream=torch.cuda.current_stream())
    torch.cuda.synchronize()
    return net.get_output_scaling()


def test_noalloc_output_scaling_matches_allocating():
    import torch
    g = torch.Generator(device="cuda").manual_seed(11)
    for rows, n_out in ((70001, 1100), (3000, 700)):     # second call: smaller input
        net = MLPm.MLP(8, 32, n_out, max_batch=64)
        y = (torch.randn(rows, n_out, device="cuda", generator=g) * 3.0 + 0.5).contiguous()
        y[:, :5] = 0.25          # constant columns: spread floored at sd_min
        m_ref, s_ref = _fit(net, y, noalloc=False)
        m, s = _fit(net, y, noalloc=True)
        assert np.array_equal(m, m_ref) and np.array_equal(s, s_ref)
        assert np.all(s[:5] == np.float32(1e-4))
        yh = y.double().cpu().numpy()
        assert np.allclose(m, yh.mean(0), rtol=1e-6, atol=1e-6)
        assert np.allclose(s, np.maximum(yh.std(0), 1e-4), rtol=1e-5)
        del net


def test_noalloc_output_scaling_rejects_oversize():
    import torch
    net = MLPm.MLP(1, 1, (1 << 19) + 1, max_batch=1)
    y = torch.zeros(2, (1 << 19) + 1, device="cuda")
    with pytest.raises(A.AdmmError) as e:
        net.fit_output_scaling_noalloc(y)
    assert e.value.status == A.E_UNSUPPORTED
