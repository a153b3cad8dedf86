"""The allocation-free forward pass of the warm-start network
(lbib_mlp_forward_noalloc) against the workspace forward pass
(lbib_mlp_forward): the same kernels on the same inputs, so the outputs are
bitwise equal.  Two calls in a row, the second with a smaller batch, then
the size limits."""
import numpy as np
import pytest

from paper_1906_03065_amd import lbib

pytestmark = pytest.mark.gpu


def test_mlp_forward_noalloc_matches_workspace_forward():
    import torch

    g = np.random.default_rng(12)
    n = lbib.lib().lbib_mlp_param_count()
    params = (g.standard_normal(n) * 0.2).astype(np.float32)
    m = lbib.Mlp(4096)
    m.set_params(params)
    dev = m.device
    pdev = torch.as_tensor(params).to(dev)
    for B in (4096, 300):
        x = g.uniform(-2.0, 2.0, (B, 6)).astype(np.float32)
        ref = m.forward(x)
        xd = torch.as_tensor(x).to(dev)
        y = torch.full((B, 32), float("nan"), dtype=torch.float32, device=dev)
        print("noalloc forward B =", B, flush=True)
        lbib.mlp_forward_noalloc(pdev, xd, y)
        torch.cuda.synchronize(dev)
        assert torch.isfinite(y).all()
        assert torch.equal(y, ref), float((y - ref).abs().max())
    x = torch.zeros((4097, 6), dtype=torch.float32, device=dev)
    y = torch.zeros((4097, 32), dtype=torch.float32, device=dev)
    with pytest.raises(lbib.LbibError) as e:
        lbib.mlp_forward_noalloc(pdev, x, y)
    assert e.value.code == lbib.ENOMEM
    st = torch.cuda.current_stream(dev).cuda_stream
    L = lbib.lib()
    assert L.lbib_mlp_forward_noalloc(pdev.data_ptr(), x.data_ptr(), 0, y.data_ptr(), st) == lbib.EINVAL
    assert L.lbib_mlp_forward_noalloc(None, x.data_ptr(), 5, y.data_ptr(), st) == lbib.EINVAL
