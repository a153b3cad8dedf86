"""FP64 reference of the warm-start network -- test infrastructure only
(only tests and the benchmark's CPU leg may use it).

A fully connected map 6 -> 128 -> 128 -> 32 with GELU(z) = z Phi(z) after the
two hidden layers, the loss sum (y - t)^2 / (2 B) over a batch of B rows,
its gradient by backpropagation written out layer by layer, and one Adam
step with bias-corrected moments.  Parameter layout (one flat array): W1
[128][6], b1 [128], W2 [128][128], b2 [128], W3 [32][128], b3 [32].
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

IN, H, OUT = 6, 128, 32
SIZES = [(H, IN), (H,), (H, H), (H,), (OUT, H), (OUT,)]
NPARAM = sum(int(np.prod(s)) for s in SIZES)


def split(p: np.ndarray) -> list:
    """Views W1, b1, W2, b2, W3, b3 of the flat parameter array."""
    out, o = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(p[o:o + n].reshape(s))
        o += n
    return out


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    """d/dz z Phi(z) = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def forward(p: np.ndarray, X: np.ndarray):
    """Network output and the pre-activations of the hidden layers."""
    W1, b1, W2, b2, W3, b3 = split(np.asarray(p, dtype=np.float64))
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    A1 = gelu(Z1)
    Z2 = A1 @ W2.T + b2
    A2 = gelu(Z2)
    Y = A2 @ W3.T + b3
    return Y, (X, Z1, A1, Z2, A2)


def loss_grad(p: np.ndarray, X: np.ndarray, T: np.ndarray):
    """(loss, gradient) with loss = sum (Y - T)^2 / (2 B)."""
    Y, (X, Z1, A1, Z2, A2) = forward(p, X)
    W1, b1, W2, b2, W3, b3 = split(np.asarray(p, dtype=np.float64))
    B = X.shape[0]
    E = Y - np.asarray(T, dtype=np.float64)
    loss = 0.5 * float((E * E).sum()) / B
    dY = E / B
    gW3 = dY.T @ A2
    gb3 = dY.sum(0)
    dZ2 = (dY @ W3) * gelu_grad(Z2)
    gW2 = dZ2.T @ A1
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2) * gelu_grad(Z1)
    gW1 = dZ1.T @ X
    gb1 = dZ1.sum(0)
    g = np.concatenate([a.reshape(-1) for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    return loss, g


def adam(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1): new parameters and moments."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
