"""Hyperelastic strain laws of a 2D ring (the paper names neo-Hookean and
Skalak membranes as alternatives to its law, eq. DiscreteSE, without
formulas).  The oracle's ring energies are pinned against the general
two-stretch membrane laws evaluated at plane strain (second stretch 1), its
forces against finite differences of its energies, and the laws against the
paper's law at small strain."""
import numpy as np
import pytest

import oracle as O
from helpers import ring_laplace, ring_law_tension, run_oracle
from paper_1906_03065_amd import workloads as W

KS = 0.037


def w_neo_hookean(l1, l2, G):
    """neo-Hookean membrane energy per reference area (incompressible 3D
    material, thickness eliminated)."""
    return 0.5 * G * (l1 ** 2 + l2 ** 2 + 1.0 / (l1 * l2) ** 2 - 3.0)


def w_skalak(l1, l2, G, C):
    I1 = l1 ** 2 + l2 ** 2 - 2.0
    I2 = (l1 * l2) ** 2 - 1.0
    return 0.25 * G * (I1 ** 2 + 2.0 * I1 - 2.0 * I2 + C * I2 ** 2)


def w_general(law, lam, C=1.0):
    """The law per unit rest length of a ring segment, from the general laws
    with the moduli that give the paper's small-strain modulus KS:
    neo-Hookean G = KS/4, Skalak G (1 + C) = KS/2."""
    if law == 0:
        return 0.5 * KS * (lam - 1.0) ** 2
    if law == 1:
        return w_neo_hookean(lam, 1.0, KS / 4.0)
    return w_skalak(lam, 1.0, KS / (2.0 * (1.0 + C)), C)


def _polygon(n=24, R=10.0):
    return W.circle_markers(0.0, 0.0, R, n)


def _rest(X):
    return np.linalg.norm(np.roll(X, -1, axis=0) - X, axis=1)


@pytest.mark.parametrize("law", [0, 1, 2])
@pytest.mark.parametrize("lam", [0.7, 0.95, 1.0, 1.1, 1.6])
def test_uniform_scaling_energy_matches_general_law(law, lam):
    X0 = _polygon()
    rest = _rest(X0)
    F, es, eb = O.ring_forces(lam * X0, rest, KS, 0.0, law=law)
    for C in (1.0, 4.0):
        assert es == pytest.approx(rest.sum() * w_general(law, lam, C), rel=1e-12, abs=1e-15)
    # every marker is pulled radially (in for lam > 1) with 2 T sin(pi / n),
    # T = dW/dlam of the general law (central difference)
    h = 1e-6
    T = (w_general(law, lam + h) - w_general(law, lam - h)) / (2 * h)
    r = lam * X0 / np.linalg.norm(X0, axis=1)[:, None] / lam
    Fr = (F * r).sum(1)
    np.testing.assert_allclose(Fr, -2.0 * T * np.sin(np.pi / len(X0)), rtol=1e-7, atol=1e-13)
    np.testing.assert_allclose(F[:, 0] * r[:, 1] - F[:, 1] * r[:, 0], 0.0, atol=1e-13)


@pytest.mark.parametrize("law", [1, 2])
def test_forces_are_minus_energy_gradient(law):
    g = np.random.default_rng(3)
    X0 = _polygon(n=17, R=8.0) + g.normal(0, 0.3, (17, 2))
    rest = _rest(X0) * g.uniform(0.8, 1.2, 17)
    X = X0 * 1.1 + g.normal(0, 0.2, X0.shape)
    F, _, _ = O.ring_forces(X, rest, KS, 2e-3, law=law)
    h = 1e-6
    for k in range(X.shape[0]):
        for a in range(2):
            Xp, Xm = X.copy(), X.copy()
            Xp[k, a] += h
            Xm[k, a] -= h
            ep = sum(O.ring_forces(Xp, rest, KS, 2e-3, law=law)[1:])
            em = sum(O.ring_forces(Xm, rest, KS, 2e-3, law=law)[1:])
            assert F[k, a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-6, abs=1e-10)


def test_laws_agree_at_small_strain():
    """Same small-strain modulus: relative differences in energy shrink in
    proportion to the strain."""
    X0 = _polygon()
    rest = _rest(X0)
    d = {}
    for eps in (1e-2, 1e-3):
        e0 = O.ring_forces((1 + eps) * X0, rest, KS, 0.0, law=0)[1]
        d[eps] = [abs(O.ring_forces((1 + eps) * X0, rest, KS, 0.0, law=l)[1] / e0 - 1.0) for l in (1, 2)]
    for k in range(2):
        assert d[1e-3][k] < 2e-3
        assert 8.0 < d[1e-2][k] / d[1e-3][k] < 12.0


def test_law_rules():
    p = W.base_params(32, 32, kappa_c=0.0)
    s = O.Sim(p)
    s.add_membrane(_polygon(n=12, R=6.0) + 16.0, None, KS, 0.0)
    for bad in (-1, 3):
        with pytest.raises(ValueError):
            s.set_membrane_law(0, bad)
    with pytest.raises(ValueError):
        s.set_membrane_law(1, 1)
    s.set_membrane_law(0, 2)
    with pytest.raises(ValueError):
        s.set_rest(0, np.zeros(12))
    s.set_rest(0, np.full(12, 3.0))


def test_hand_derivatives_of_the_general_laws():
    """The tensions used by the Laplace checks against central differences of
    the general laws."""
    h = 1e-6
    for law in (0, 1, 2):
        for lam in (0.8, 1.25, 1.5):
            fd = (w_general(law, lam + h) - w_general(law, lam - h)) / (2 * h)
            assert ring_law_tension(law, KS, lam) == pytest.approx(fd, rel=1e-7)


@pytest.mark.parametrize("law", [0, 1, 2])
def test_prestressed_ring_laplace_law(law):
    """A ring stretched by 1.25 in a uniform fluid settles where the pressure
    jump balances its tension, dp = T(lam)/R (2D Laplace law of a membrane
    under tension), for each strain law; T differs by 30-40 % between the
    laws at this stretch."""
    w = W.prestressed_ring(law)
    o = run_oracle(O, w)
    o.step(6000)
    dp, pred = ring_laplace(o, w)
    assert dp == pytest.approx(pred, rel=3e-3), (dp, pred)


# ---- 3D meshes: the laws per triangle, shear modulus KS, Skalak C = 1 ----

def _mesh(subdiv=1, R=6.0):
    V, T = W.icosphere(subdiv)
    return R * V, T


def _edge_rest(V, T):
    """Rest lengths in the oracle's edge order (first appearance over the
    triangles' edges (v_k, v_k+1)), from the rest configuration V."""
    seen, rest = {}, []
    for t in T:
        for k in range(3):
            a, b = int(t[k]), int(t[(k + 1) % 3])
            key = (min(a, b), max(a, b))
            if key not in seen:
                seen[key] = len(rest)
                rest.append(np.linalg.norm(V[a] - V[b]))
    return np.array(rest)


def _energy_by_svd(V0, X, T, law):
    """Sum over triangles of A0 W(l1, l2): the principal stretches l1, l2
    are the singular values of the in-plane linear map from the rest
    triangle to the current one, and W the general membrane law."""
    E = 0.0
    for t in T:
        P0, P = V0[t], X[t]
        E0 = np.stack([P0[1] - P0[0], P0[2] - P0[0]], axis=1)  # 3 x 2
        E1 = np.stack([P[1] - P[0], P[2] - P[0]], axis=1)
        M = E1 @ np.linalg.pinv(E0)                              # maps the rest plane onto the current one
        s = np.linalg.svd(M, compute_uv=False)[:2]
        A0 = 0.5 * np.linalg.norm(np.cross(E0[:, 0], E0[:, 1]))
        w = w_neo_hookean(s[0], s[1], KS) if law == 1 else w_skalak(s[0], s[1], KS, 1.0)
        E += A0 * w
    return E


@pytest.mark.parametrize("law", [1, 2])
def test_mesh_laws_against_principal_stretches(law):
    """Equibiaxial scaling and an anisotropic, sheared deformation of an
    icosphere: the oracle's energy equals the SVD-based sum."""
    V0, T = _mesh()
    rest = _edge_rest(V0, T)
    g = np.random.default_rng(7)
    A = np.array([[1.3, 0.2, 0.0], [0.0, 0.9, 0.1], [0.05, 0.0, 1.1]])
    for X in (1.2 * V0, V0 @ A.T, V0 @ A.T + g.normal(0, 0.05, V0.shape)):
        _, es, _ = O.mesh_forces(X, T, rest, KS, 0.0, law=law)
        assert es == pytest.approx(_energy_by_svd(V0, X, T, law), rel=1e-10)
    # at rest the neo-Hookean and Skalak energies vanish
    assert abs(O.mesh_forces(V0, T, rest, KS, 0.0, law=law)[1]) < 1e-12


@pytest.mark.parametrize("law", [1, 2])
def test_mesh_law_forces_are_minus_energy_gradient(law):
    V0, T = _mesh()
    rest = _edge_rest(V0, T)
    g = np.random.default_rng(8)
    X = 1.1 * V0 + g.normal(0, 0.1, V0.shape)
    F, _, _ = O.mesh_forces(X, T, rest, KS, 1e-3, law=law)
    h = 1e-6
    for v in range(0, len(V0), 5):
        for a in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[v, a] += h
            Xm[v, a] -= h
            ep = sum(O.mesh_forces(Xp, T, rest, KS, 1e-3, law=law)[1:])
            em = sum(O.mesh_forces(Xm, T, rest, KS, 1e-3, law=law)[1:])
            assert F[v, a] == pytest.approx(-(ep - em) / (2 * h), rel=1e-6, abs=1e-11)
    # a closed membrane's internal forces sum to zero
    np.testing.assert_allclose(F.sum(0), 0.0, atol=1e-13)
