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
