"""The sharp-interface reference for the capsule-at-interface shapes
(oracle/sharp.py, standing in for the paper's finite-element comparisons of
Sec. 3.4): its energy gradient against finite differences, its liquid-lens
limit against the closed form from Neumann's triangle (eq. SurfaceTension
tensions), the mirror symmetry of the symmetric case, and the Taylor
deformation measure on ellipses."""
import numpy as np
import pytest

from oracle import sharp as S
from paper_1906_03065_amd import taylor as T
from paper_1906_03065_amd import workloads as W


def _model(kappa, ks, kb, n=64, R=20.0):
    X0 = W.circle_markers(120.0, 59.5, R, n)
    rest = np.linalg.norm(np.roll(X0, -1, axis=0) - X0, axis=1)
    g12, g13, g23 = S.tensions(kappa, 2.0)
    return S.CapsuleAtInterface(X0, rest, ks, kb, g12, g13, g23, (0.0, 59.5), (240.0, 59.5))


def lens_closed_form(g12, g13, g23, area):
    """A lens of fluid 3 between fluid 1 (below) and fluid 2 (above): two
    circular caps on a flat chord, meeting it at angles b1 (lower) and b2
    (upper) with g12 = g13 cos b1 + g23 cos b2 and g13 sin b1 = g23 sin b2.
    A cap on a half-chord a with angle b has radius a / sin b and area
    a^2 (b - sin b cos b) / sin^2 b; the caps' areas add up to `area`.
    Returns D = (L - B)/(L + B) with L, B the chord and the total height."""
    b1 = np.arccos((g12 ** 2 + g13 ** 2 - g23 ** 2) / (2 * g12 * g13))
    b2 = np.arcsin(g13 * np.sin(b1) / g23)
    f = lambda b: (b - np.sin(b) * np.cos(b)) / np.sin(b) ** 2
    a = np.sqrt(area / (f(b1) + f(b2)))
    h = a * (1 - np.cos(b1)) / np.sin(b1) + a * (1 - np.cos(b2)) / np.sin(b2)
    L, B = max(2 * a, h), min(2 * a, h)
    return (L - B) / (L + B)


def test_energy_gradient():
    m = _model((8e-3, 2e-3, 3e-3), 1e-2, 1e-3, n=24, R=8.0)
    g = np.random.default_rng(1)
    z = m.initial()
    z[:-2] += g.normal(0, 0.2, z.size - 2)
    z[-2:] += (0.3, -0.4)
    E, G = m.energy(z)
    h = 1e-6
    for i in range(z.size):
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        fd = (m.energy(zp)[0] - m.energy(zm)[0]) / (2 * h)
        assert G[i] == pytest.approx(fd, rel=1e-6, abs=1e-10), i


@pytest.mark.parametrize("kappa", [(8e-3, 8e-3, 5e-4), (8e-3, 2e-3, 5e-4)])
def test_liquid_lens_limit(kappa):
    """Without membrane energies (a vanishing strain modulus keeps the
    markers spread) the capsule is a liquid lens: D within 1e-3 of the closed
    form, the area conserved."""
    m = _model(kappa, 1e-7, 0.0)
    X, _, _, r = m.solve(maxiter=6000)
    g12, g13, g23 = m.g12, m.g13, m.g23
    D = S.taylor_deformation(X)
    assert D == pytest.approx(lens_closed_form(g12, g13, g23, m.area0), rel=1e-3)
    assert S.polygon_area(X)[0] == pytest.approx(m.area0, rel=1e-12)


def test_symmetric_case_contact_points():
    """Equal tensions g13 = g23: the contact points stay on the interface
    height, mirror images about the box centre, and the fluid-fluid lines are
    horizontal.  (The capsule itself may settle a little off-centre in y:
    the discrete model has two mirror-image minima there.)"""
    m = _model((8e-3, 8e-3, 2e-3), 1e-2, 1e-4)
    X, uL, uR, r = m.solve()
    assert r.success
    CL, CR = S.point(X, uL)[0], S.point(X, uR)[0]
    for C in (CL, CR):
        assert C[1] == pytest.approx(59.5, abs=1e-4)
    assert CL[0] + CR[0] == pytest.approx(240.0, abs=1e-3)


@pytest.mark.parametrize("measure", [S.taylor_deformation, T.taylor_deformation])
@pytest.mark.parametrize("a,b,rot", [(30.0, 10.0, 0.0), (12.0, 9.0, 0.7), (20.0, 20.0, 0.3)])
def test_taylor_deformation_of_ellipses(measure, a, b, rot):
    t = 2 * np.pi * np.arange(2000) / 2000
    P = np.stack([a * np.cos(t), b * np.sin(t)], axis=1)
    c, s = np.cos(rot), np.sin(rot)
    X = P @ np.array([[c, s], [-s, c]]) + (50.0, -7.0)
    assert measure(X) == pytest.approx((a - b) / (a + b), abs=1e-5)
