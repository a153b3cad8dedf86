"""The warm-start network's HIP kernels against the FP64 reference:
forward pass, loss gradient (relative error <= 1e-4), the Adam update, and
that training lowers the loss."""
import numpy as np
import pytest

from oracle import mlp_ref as M
from paper_1906_03065_amd import lbib, mlp

pytestmark = pytest.mark.gpu


def _data(B, seed):
    g = np.random.default_rng(seed)
    X = g.normal(size=(B, 6)).astype(np.float32)
    T = g.normal(size=(B, 32)).astype(np.float32)
    return X, T


@pytest.mark.parametrize("B", [1, 37, 300, 4096])
def test_forward_and_gradient_vs_fp64(B):
    """Ragged and full batch sizes (tiles of 64 rows plus a tail)."""
    p = mlp.init_params(5)
    p[M.NPARAM - 32:] = 0.1  # non-zero output bias
    X, T = _data(B, B)
    net = lbib.Mlp(4096)
    net.set_params(p)
    y = net.forward(X).cpu().numpy()
    yo, _ = M.forward(p.astype(np.float64), X.astype(np.float64))
    ey = np.abs(y - yo).max() / np.abs(yo).max()
    loss, g = net.gradient(X, T)
    lo, go = M.loss_grad(p.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    eg = np.abs(g - go).max() / np.abs(go).max()
    print(B, "forward", ey, "grad", eg, "loss", loss, lo, flush=True)
    assert ey < 1e-5
    assert eg < 1e-4
    assert abs(loss / lo - 1) < 1e-5
    # every layer separately
    offs = np.cumsum([0] + [int(np.prod(s)) for s in M.SIZES])
    for k in range(6):
        a, b = offs[k], offs[k + 1]
        assert np.abs(g[a:b] - go[a:b]).max() <= 1e-4 * max(np.abs(go[a:b]).max(), 1e-6 * np.abs(go).max()), k


def test_adam_step_vs_fp64():
    """Three Adam steps on the device equal three reference steps taken
    with the device's own gradients (FP32 rounding only)."""
    p = mlp.init_params(6)
    X, T = _data(256, 7)
    net = lbib.Mlp(256)
    net.set_params(p)
    ref = p.astype(np.float64)
    m = np.zeros(M.NPARAM)
    v = np.zeros(M.NPARAM)
    for t in range(1, 4):
        _, g = net.gradient(X, T)
        net.adam_step(X, T, lr=1e-2)
        ref, m, v = M.adam(ref, g.astype(np.float64), m, v, t, lr=1e-2)
        dev = net.params()
        assert np.abs(dev - ref).max() < 1e-5, t


def test_training_lowers_loss():
    """Fit a smooth map of the six inputs: the loss falls by two orders."""
    g = np.random.default_rng(8)
    X = g.uniform(-1, 1, size=(1024, 6))
    A = g.normal(size=(6, 32))
    Y = np.tanh(X @ A) + 0.1 * np.sin(3 * X[:, :1])
    model, hist = mlp.train(X, Y, epochs=600, lr=3e-3, log_every=100)
    print(hist, flush=True)
    assert hist[-1][1] < 0.01 * hist[0][1]
    pred = model.predict(X[:200])
    rms = np.sqrt(((pred - Y[:200]) ** 2).mean(0)) / Y.std(0)
    print("rms / std per output", rms.max(), flush=True)
    assert rms.max() < 0.25 and rms.mean() < 0.15
