"""Shape coefficients of a 2D capsule and their inverse (host side).

A closed marker polygon is described by 32 numbers: the vertical offset of
its area centroid from a reference height, over R, and the radial Fourier
series of r(theta)/R about the centroid, a_0..a_15 and b_1..b_15.  The
series is a least-squares fit to the markers' polar coordinates.  The
inverse places n markers at equal arc-length fractions of the curve (dense
sampling of r(theta), then arc-length interpolation), counter-clockwise
starting at the angle pi/n.

Also the equilibrium criterion used for "steps to equilibrium": every 100
steps, the largest marker speed below 1e-6 and the coefficients changed by
less than 1e-4 R over the last 1000 steps.
"""
from __future__ import annotations

import numpy as np

K = 16  # cosine terms a_0..a_15, sine terms b_1..b_15
NCOEF = 1 + K + (K - 1)


def centroid(X: np.ndarray) -> np.ndarray:
    """Area centroid of a simple polygon (rows x, y)."""
    x, y = X[:, 0], X[:, 1]
    x1, y1 = np.roll(x, -1), np.roll(y, -1)
    c = x * y1 - x1 * y
    A = 0.5 * c.sum()
    return np.array([((x + x1) * c).sum() / (6 * A), ((y + y1) * c).sum() / (6 * A)])


def _basis(theta: np.ndarray) -> np.ndarray:
    cols = [np.cos(k * theta) for k in range(K)] + [np.sin(k * theta) for k in range(1, K)]
    return np.stack(cols, axis=1)


def coefficients(X: np.ndarray, R: float, y_ref: float) -> np.ndarray:
    """[dy_c/R, a_0..a_15, b_1..b_15] of marker polygon X."""
    c = centroid(X)
    d = X - c
    theta = np.arctan2(d[:, 1], d[:, 0])
    r = np.hypot(d[:, 0], d[:, 1]) / R
    coef, *_ = np.linalg.lstsq(_basis(theta), r, rcond=None)
    return np.concatenate([[(c[1] - y_ref) / R], coef])


def curve(coef: np.ndarray, R: float, centre: np.ndarray, m: int = 4096) -> np.ndarray:
    """Dense samples of the curve r(theta) about centre (m points)."""
    theta = np.linspace(0.0, 2 * np.pi, m, endpoint=False)
    r = R * (_basis(theta) @ coef[1:])
    return np.stack([centre[0] + r * np.cos(theta), centre[1] + r * np.sin(theta)], axis=1)


def markers(coef: np.ndarray, R: float, x_c: float, y_ref: float, n: int) -> np.ndarray:
    """n markers at equal arc-length fractions of the curve given by coef,
    its centroid at (x_c, y_ref + dy_c R), counter-clockwise."""
    centre = np.array([x_c, y_ref + coef[0] * R])
    P = curve(coef, R, centre)
    Pc = np.vstack([P, P[:1]])
    seg = np.hypot(*np.diff(Pc, axis=0).T)
    s = np.concatenate([[0.0], np.cumsum(seg)])
    t = (np.arange(n) + 0.5) / n * s[-1]
    X = np.stack([np.interp(t, s, Pc[:, 0]), np.interp(t, s, Pc[:, 1])], axis=1)
    # the sampled curve's centroid differs slightly from the requested one
    return X + (centre - centroid(X))


def signed_distance(X: np.ndarray, px: np.ndarray, py: np.ndarray) -> np.ndarray:
    """Signed distance of points (px, py) to polygon X, positive inside
    (for building initial concentration fields)."""
    A = X
    B = np.roll(X, -1, axis=0)
    best = np.full(px.shape, np.inf)
    inside = np.zeros(px.shape, dtype=bool)
    for a, b in zip(A, B):
        e = b - a
        t = np.clip(((px - a[0]) * e[0] + (py - a[1]) * e[1]) / (e @ e), 0.0, 1.0)
        d = np.hypot(px - a[0] - t * e[0], py - a[1] - t * e[1])
        best = np.minimum(best, d)
        cross = (a[1] > py) != (b[1] > py)
        xc = a[0] + (py - a[1]) * e[0] / np.where(e[1] == 0, 1.0, e[1])
        inside ^= cross & (px < xc)
    return np.where(inside, best, -best)


class Equilibrium:
    """Tracks the equilibrium criterion of one capsule from samples taken
    every `every` steps (marker speeds and coefficients)."""

    def __init__(self, R: float, every: int = 100, window: int = 1000, u_tol: float = 1e-6,
                 c_tol: float = 1e-4):
        self.R, self.every, self.window = R, every, window
        self.u_tol, self.c_tol = u_tol, c_tol
        self.hist = []  # (step, coefficients)
        self.reached_at = None

    def update(self, step: int, U: np.ndarray, coef: np.ndarray) -> bool:
        self.hist.append((step, coef))
        old = [c for s, c in self.hist if s <= step - self.window]
        if self.reached_at is None and old:
            umax = float(np.abs(U).max())
            dc = float(np.abs(coef - old[-1]).max()) * self.R
            if umax < self.u_tol and dc < self.c_tol * self.R:
                self.reached_at = step
        # keep what the window needs
        self.hist = [(s, c) for s, c in self.hist if s > step - self.window - self.every]
        return self.reached_at is not None
