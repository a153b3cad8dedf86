"""Pins of the FP64 reference of the warm-start network: GELU against the
normal distribution function, the backpropagated gradient against central
finite differences of the loss, a network that reduces to its output bias,
and the closed form of the first Adam step."""
import math

import numpy as np

from oracle import mlp_ref as M


def _params(seed, scale=0.3):
    g = np.random.default_rng(seed)
    return g.normal(scale=scale, size=M.NPARAM)


def test_gelu_values():
    """GELU(z) = z Phi(z): zero at zero, GELU(z) - GELU(-z) = z (Phi(z) +
    Phi(-z) = 1), and Phi(3) = 0.998650101968 (normal table)."""
    z = np.linspace(-4, 4, 81)
    assert M.gelu(np.array(0.0)) == 0.0
    np.testing.assert_allclose(M.gelu(z) - M.gelu(-z), z, atol=1e-15)
    assert abs(M.gelu(np.array(3.0)) - 3 * 0.998650101968) < 1e-11
    h = 1e-6
    np.testing.assert_allclose(M.gelu_grad(z), (M.gelu(z + h) - M.gelu(z - h)) / (2 * h), atol=1e-9)


def test_gradient_matches_finite_differences():
    """Backpropagation against central differences of the loss on a sample
    of parameters from every layer (weights and biases)."""
    g = np.random.default_rng(1)
    p = _params(2)
    X = g.normal(size=(5, M.IN))
    T = g.normal(size=(5, M.OUT))
    _, grad = M.loss_grad(p, X, T)
    offs = np.cumsum([0] + [int(np.prod(s)) for s in M.SIZES])
    idx = np.concatenate([g.choice(np.arange(offs[k], offs[k + 1]), size=min(40, offs[k + 1] - offs[k]),
                                   replace=False) for k in range(6)])
    h = 1e-6
    fd = []
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd.append((M.loss_grad(pp, X, T)[0] - M.loss_grad(pm, X, T)[0]) / (2 * h))
    fd = np.array(fd)
    assert np.abs(grad[idx] - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def test_output_bias_only_network():
    """With every weight zero the output is b3 for every row, the loss is
    sum (b3 - t)^2 / (2B) and only b3 gets a gradient: mean over rows of
    (b3 - t)."""
    p = np.zeros(M.NPARAM)
    b3 = np.linspace(-1, 1, M.OUT)
    p[-M.OUT:] = b3
    g = np.random.default_rng(3)
    X = g.normal(size=(7, M.IN))
    T = g.normal(size=(7, M.OUT))
    Y, _ = M.forward(p, X)
    np.testing.assert_array_equal(Y, np.broadcast_to(b3, Y.shape))
    loss, grad = M.loss_grad(p, X, T)
    assert abs(loss - 0.5 * ((b3 - T) ** 2).sum() / 7) < 1e-14
    np.testing.assert_allclose(grad[-M.OUT:], (b3 - T).mean(0), atol=1e-15)
    # GELU(0) = 0 and the zero weights leave every other gradient zero
    # except W3's, which sees zero activations, and b1, b2, which see W = 0
    assert np.abs(grad[:-M.OUT]).max() == 0.0


def test_adam_first_step_closed_form():
    """First step: the bias-corrected moments are g and g^2, so the update
    is -lr g / (|g| + eps)."""
    g = np.array([1e-3, -2.0, 0.5, 0.0])
    p0 = np.array([1.0, 2.0, 3.0, 4.0])
    p1, m, v = M.adam(p0, g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    np.testing.assert_allclose(p1, p0 - 0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_param_count():
    assert M.NPARAM == 128 * 6 + 128 + 128 * 128 + 128 + 32 * 128 + 32 == 21536
    assert math.isclose(float(M.gelu(np.array(1.0))), 0.5 * (1 + math.erf(1 / math.sqrt(2))))
