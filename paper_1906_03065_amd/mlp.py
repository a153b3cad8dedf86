"""Training and use of the warm-start network (device work in the library's
hand-written kernels through lbib.Mlp).

Inputs and outputs are standardised with the training set's mean and
standard deviation; the parameters start from a seeded uniform draw in
+-1/sqrt(fan_in) (biases zero) and are trained full batch with Adam.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbib

IN, H, OUT = 6, 128, 32


def init_params(seed: int = 0) -> np.ndarray:
    g = np.random.default_rng(seed)
    parts = []
    for fan_out, fan_in in ((H, IN), (H, H), (OUT, H)):
        a = 1.0 / math.sqrt(fan_in)
        parts.append(g.uniform(-a, a, size=fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


class WarmStartModel:
    """Standardisation + network parameters; predict() maps raw features
    [B][6] to raw shape coefficients [B][32]."""

    def __init__(self, params, x_mean, x_std, y_mean, y_std):
        self.params = np.asarray(params, dtype=np.float32)
        self.x_mean, self.x_std = np.asarray(x_mean), np.asarray(x_std)
        self.y_mean, self.y_std = np.asarray(y_mean), np.asarray(y_std)

    def save(self, path: str):
        np.savez(path, params=self.params, x_mean=self.x_mean, x_std=self.x_std, y_mean=self.y_mean,
                 y_std=self.y_std)

    @classmethod
    def load(cls, path: str) -> "WarmStartModel":
        d = np.load(path)
        return cls(d["params"], d["x_mean"], d["x_std"], d["y_mean"], d["y_std"])

    def predict(self, X: np.ndarray, device="cuda:0") -> np.ndarray:
        X = np.asarray(X, dtype=np.float64)
        net = lbib.Mlp(max(1, len(X)), device=device)
        net.set_params(self.params)
        y = net.forward((X - self.x_mean) / self.x_std).cpu().numpy().astype(np.float64)
        net.close()
        return y * self.y_std + self.y_mean


def train(X: np.ndarray, Y: np.ndarray, epochs: int = 4000, lr: float = 2e-3, seed: int = 0,
          device="cuda:0", log_every: int = 500):
    """Full-batch Adam on standardised data; returns (model, loss history)."""
    import torch

    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    xm, xs = X.mean(0), X.std(0) + 1e-12
    ym, ys = Y.mean(0), Y.std(0) + 1e-12
    net = lbib.Mlp(len(X), device=device)
    net.set_params(init_params(seed))
    xd = torch.as_tensor(((X - xm) / xs).astype(np.float32), device=device)
    yd = torch.as_tensor(((Y - ym) / ys).astype(np.float32), device=device)
    hist = []
    for ep in range(epochs):
        # step size decays by 10x over the run (cosine)
        lr_e = lr * (0.1 + 0.9 * 0.5 * (1 + math.cos(math.pi * ep / epochs)))
        want = ep % log_every == 0 or ep == epochs - 1
        loss = net.adam_step(xd, yd, lr=lr_e, want_loss=want)
        if want:
            hist.append((ep, loss))
    model = WarmStartModel(net.params(), xm, xs, ym, ys)
    net.close()
    return model, hist
