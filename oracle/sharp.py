"""Sharp-interface equilibrium of a 2D capsule at a fluid-fluid interface.

Test infrastructure (a reference for the diffuse-interface simulations, like
the finite-element model of the paper's Sec. 3.4): not part of the product
path.  The paper compares its capsule shapes with a sharp-interface model in
which the interfaces are lines carrying their tension, the membrane carries
the discrete strain and bending energies of eqs. DiscreteSE and DiscreteBE,
the capsule's area is conserved, and the ends of the fluid-fluid interface
are held at the box edges.  This module minimises that energy with SLSQP:

    E = E_s(X) + E_b(X) + g23 |upper arc| + g13 |lower arc|
        + g12 (|C_L - A_L| + |C_R - A_R|),   area(X) = area(X_0)

X are the capsule markers (a closed polygon), C_L and C_R the two points
where the fluid 1 | fluid 2 interface meets the membrane.  They slide freely
along the polygon (READING: the diffuse interface is not pinned to membrane
material points), parametrised by u in [0, n): segment floor(u) at fraction
u - floor(u).  The upper arc runs counter-clockwise from C_R to C_L and is
wetted by fluid 2 (above), the lower arc by fluid 1.  A_L, A_R are the fixed
ends (box edges at the interface height).  Tensions g_mn = alpha (kappa_m +
kappa_n) / 6 (eq. SurfaceTension).
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import minimize

from . import ring_forces


def tensions(kappa, alpha):
    k1, k2, k3 = kappa
    return alpha * (k1 + k2) / 6.0, alpha * (k1 + k3) / 6.0, alpha * (k2 + k3) / 6.0


def _seg(X, k):
    n = len(X)
    return X[k % n], X[(k + 1) % n]


def point(X, u):
    """Point of the polygon at parameter u, its segment and fraction."""
    n = len(X)
    u = u % n
    k = int(np.floor(u))
    t = u - k
    a, b = _seg(X, k)
    return a + t * (b - a), k, t


def arc(X, u1, u2):
    """Length of the polygon counter-clockwise from u1 to u2, and its gradient
    with respect to X (n x 2), u1 and u2."""
    n = len(X)
    u1, u2 = u1 % n, u2 % n
    d = (u2 - u1) % n
    k1, t1 = int(np.floor(u1)), u1 - np.floor(u1)
    G = np.zeros_like(X)
    L = 0.0

    def add(k, w):
        nonlocal L
        a, b = _seg(X, k)
        e = b - a
        le = np.hypot(e[0], e[1])
        L += w * le
        G[(k + 1) % n] += w * e / le
        G[k % n] -= w * e / le
        return le

    if t1 + d <= 1.0:  # both ends on segment k1
        le = add(k1, d)
        return L, G, -le, le
    le1 = add(k1, 1.0 - t1)
    rest = d - (1.0 - t1)
    k = k1 + 1
    while rest > 1.0:
        add(k, 1.0)
        rest -= 1.0
        k += 1
    le2 = add(k, rest)
    return L, G, -le1, le2


def polygon_area(X):
    x, y = X[:, 0], X[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    A = 0.5 * np.sum(x * yn - xn * y)
    G = np.stack([0.5 * (yn - np.roll(y, 1)), 0.5 * (np.roll(x, 1) - xn)], axis=1)
    return A, G


class CapsuleAtInterface:
    """The sharp-interface energy of one configuration and its minimiser."""

    def __init__(self, X0, rest, kappa_s, kappa_b, g12, g13, g23, A_L, A_R, law=0):
        self.X0 = np.asarray(X0, dtype=np.float64).copy()
        self.n = len(self.X0)
        self.rest = np.asarray(rest, dtype=np.float64)
        self.ks, self.kb, self.law = float(kappa_s), float(kappa_b), int(law)
        self.g12, self.g13, self.g23 = float(g12), float(g13), float(g23)
        self.A_L, self.A_R = np.asarray(A_L, dtype=np.float64), np.asarray(A_R, dtype=np.float64)
        self.area0 = polygon_area(self.X0)[0]

    def energy(self, z):
        """E and dE/dz for z = [X (2n), u_L, u_R]."""
        n = self.n
        X = z[:2 * n].reshape(n, 2)
        uL, uR = z[2 * n], z[2 * n + 1]
        F, es, eb = ring_forces(X, self.rest, self.ks, self.kb, law=self.law)
        E = es + eb
        G = -F
        gu = np.zeros(2)
        # upper arc C_R -> C_L (fluid 2), lower arc C_L -> C_R (fluid 1)
        Lu, Gu, du_R, du_L = arc(X, uR, uL)
        Ll, Gl, dl_L, dl_R = arc(X, uL, uR)
        E += self.g23 * Lu + self.g13 * Ll
        G += self.g23 * Gu + self.g13 * Gl
        gu[0] += self.g23 * du_L + self.g13 * dl_L
        gu[1] += self.g23 * du_R + self.g13 * dl_R
        for j, (u, A) in enumerate(((uL, self.A_L), (uR, self.A_R))):
            C, k, t = point(X, u)
            v = C - A
            lv = np.hypot(v[0], v[1])
            E += self.g12 * lv
            nv = v / lv
            G[k % n] += self.g12 * (1.0 - t) * nv
            G[(k + 1) % n] += self.g12 * t * nv
            a, b = _seg(X, k)
            gu[j] += self.g12 * float(nv @ (b - a))
        return E, np.concatenate([G.ravel(), gu])

    def initial(self):
        """Contact points at the polygon's leftmost and rightmost crossings of
        the interface height (the initial circle is centred on it)."""
        y0 = self.A_L[1]
        n = self.n
        cand = []
        for k in range(n):
            a, b = _seg(self.X0, k)
            if (a[1] - y0) * (b[1] - y0) <= 0 and a[1] != b[1]:
                t = (y0 - a[1]) / (b[1] - a[1])
                cand.append((a[0] + t * (b[0] - a[0]), k + t))
        cand.sort()
        return np.concatenate([self.X0.ravel(), [cand[0][1], cand[-1][1]]])

    def solve(self, z0=None, tol=1e-12, maxiter=5000):
        z0 = self.initial() if z0 is None else z0
        n = self.n
        cons = {"type": "eq",
                "fun": lambda z: polygon_area(z[:2 * n].reshape(n, 2))[0] - self.area0,
                "jac": lambda z: np.concatenate([polygon_area(z[:2 * n].reshape(n, 2))[1].ravel(), [0.0, 0.0]])}
        r = minimize(self.energy, z0, jac=True, method="SLSQP", constraints=[cons],
                     options={"ftol": tol, "maxiter": maxiter})
        self.result = r
        return r.x[:2 * n].reshape(n, 2), r.x[2 * n], r.x[2 * n + 1], r


def taylor_deformation(X):
    """D = (L - B) / (L + B), L and B the extents of the polygon along the
    principal axes of its second moment of area."""
    X = np.asarray(X, dtype=np.float64)[:, :2]
    x, y = X[:, 0], X[:, 1]
    xn, yn = np.roll(x, -1), np.roll(y, -1)
    cr = x * yn - xn * y
    A = 0.5 * cr.sum()
    cx = ((x + xn) * cr).sum() / (6 * A)
    cy = ((y + yn) * cr).sum() / (6 * A)
    xs, ys = x - cx, y - cy
    xsn, ysn = np.roll(xs, -1), np.roll(ys, -1)
    c2 = xs * ysn - xsn * ys
    Ixx = ((ys ** 2 + ys * ysn + ysn ** 2) * c2).sum() / 12
    Iyy = ((xs ** 2 + xs * xsn + xsn ** 2) * c2).sum() / 12
    Ixy = ((xs * ysn + 2 * xs * ys + 2 * xsn * ysn + xsn * ys) * c2).sum() / 24
    w, V = np.linalg.eigh(np.array([[Iyy, Ixy], [Ixy, Ixx]]))
    P = np.stack([xs, ys], axis=1) @ V
    ext = P.max(0) - P.min(0)
    L, B = ext.max(), ext.min()
    return (L - B) / (L + B)
