"""Pins of the oracle's building blocks against what the paper and the
mathematics fix (no GPU).  Each test names the passage it checks."""
import json
import os

import numpy as np
import pytest

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
CS2 = 1.0 / 3.0


def test_d2q9_tables_match_paper(orc):
    """Sec. 3.1 prints the D2Q9 velocities and weights."""
    c, w = orc.lattice(0)
    g = GOLD["d2q9"]
    assert list(c[:, 0]) == g["cx"] and list(c[:, 1]) == g["cy"] and not c[:, 2].any()
    np.testing.assert_allclose(w, g["w"], rtol=0, atol=1e-16)


@pytest.mark.parametrize("kind", [0, 1])
def test_lattice_isotropy(orc, kind):
    """Weights reproduce the moments of a Maxwellian up to fourth order
    (c_s^2 = 1/3, Sec. 3.1): sum w = 1, odd moments vanish, sum w c c = c_s^2 I,
    sum w c c c c = c_s^4 (d d + d d + d d)."""
    c, w = orc.lattice(kind)
    D = 2 if kind == 0 else 3
    c = c[:, :D].astype(float)
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs(w @ c).max() < 1e-16
    np.testing.assert_allclose(np.einsum("i,ia,ib->ab", w, c, c), CS2 * np.eye(D), atol=1e-16)
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-16
    m4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    I = np.eye(D)
    ref = CS2 ** 2 * (np.einsum("ab,cd->abcd", I, I) + np.einsum("ac,bd->abcd", I, I) +
                      np.einsum("ad,bc->abcd", I, I))
    np.testing.assert_allclose(m4, ref, atol=1e-16)
    # every velocity has its opposite
    for ci in c:
        assert any((cj == -ci).all() for cj in c)


@pytest.mark.parametrize("kind", [0, 1])
def test_feq_moments(orc, kind):
    """eq. EDF: sum f^eq = rho, sum c f^eq = rho u, sum c c f^eq = rho c_s^2 I + rho u u."""
    c, w = orc.lattice(kind)
    D = 2 if kind == 0 else 3
    c = c[:, :D].astype(float)
    g = np.random.default_rng(1)
    for _ in range(5):
        rho = g.uniform(0.8, 1.2)
        u = g.uniform(-0.1, 0.1, D)
        f = orc.feq(kind, rho, u)
        assert abs(f.sum() - rho) < 1e-14
        np.testing.assert_allclose(f @ c, rho * u, atol=1e-15)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", f, c, c),
                                   rho * CS2 * np.eye(D) + rho * np.outer(u, u), atol=1e-15)


@pytest.mark.parametrize("kind", [0, 1])
def test_geq_moments(orc, kind):
    """eq. EDF for g, h: zeroth moment q (rest population closes it), first
    moment q v, second moment Gamma mu I + q v v."""
    c, w = orc.lattice(kind)
    D = 2 if kind == 0 else 3
    c = c[:, :D].astype(float)
    g = np.random.default_rng(2)
    for _ in range(5):
        q = g.uniform(-1, 1)
        mu = g.uniform(-0.01, 0.01)
        Gam = g.uniform(0.1, 2.0)
        v = g.uniform(-0.05, 0.05, D)
        e = orc.geq(kind, q, mu, Gam, v)
        assert abs(e.sum() - q) < 1e-15
        np.testing.assert_allclose(e @ c, q * v, atol=1e-15)
        np.testing.assert_allclose(np.einsum("i,ia,ib->ab", e, c, c),
                                   Gam * mu * np.eye(D) + q * np.outer(v, v), atol=1e-15)


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("taus", [(1.0, 1.0, 1.0), (0.8, 1.3, 0.9)])
def test_collision_invariants(orc, kind, taus):
    """eq. LBE: BGK keeps the zeroth moments of f, g, h; the exact-difference
    term adds exactly the force to the momentum (eq. VelCorrection).  At
    tau = 1 the post-collision f is f^eq(rho, u + F/rho) and g, h are their
    equilibria at v = u + F/(2 rho)."""
    c, w = orc.lattice(kind)
    D = 2 if kind == 0 else 3
    cc = c[:, :D].astype(float)
    g = np.random.default_rng(3)
    p = dict(lattice=kind, nx=4, ny=4, nz=4 if kind else 1, tau=taus[0], tau_phi=taus[1],
             tau_psi=taus[2], gamma_phi=0.3, gamma_psi=0.7, kappa=[0.02, 0.03, 0.01], alpha=1.0)
    for _ in range(4):
        rho = g.uniform(0.9, 1.1)
        u = g.uniform(-0.05, 0.05, D)
        f = orc.feq(kind, rho, u) * (1 + g.uniform(-0.05, 0.05, len(w)))
        gg = orc.geq(kind, 0.3, 0.001, 1.0, u) + g.uniform(-1e-3, 1e-3, len(w))
        hh = orc.geq(kind, 0.6, -0.002, 1.0, u) + g.uniform(-1e-3, 1e-3, len(w))
        F = g.uniform(-1e-3, 1e-3, D)
        mphi, mpsi = 0.004, -0.003
        f2, g2, h2 = orc.collide(p, (f, gg, hh), F, mphi, mpsi)
        assert abs(f2.sum() - f.sum()) < 1e-14
        np.testing.assert_allclose(f2 @ cc, f @ cc + F, atol=1e-15)
        assert abs(g2.sum() - gg.sum()) < 1e-14 and abs(h2.sum() - hh.sum()) < 1e-14
        if taus == (1.0, 1.0, 1.0):
            r = f.sum()
            uu = f @ cc / r
            np.testing.assert_allclose(f2, orc.feq(kind, r, uu + F / r), atol=1e-15)
            v = uu + 0.5 * F / r
            np.testing.assert_allclose(g2, orc.geq(kind, gg.sum(), mphi, 0.3, v), atol=1e-15)
            np.testing.assert_allclose(h2, orc.geq(kind, hh.sum(), mpsi, 0.7, v), atol=1e-15)


def test_peskin_kernel(orc):
    """eq. DiscreteDirac (Peskin 4-point): partition of unity, zero first
    moment, sum of squares 3/8, even and odd sums 1/2, support |r| < 2."""
    g = np.random.default_rng(4)
    for r in g.uniform(0, 1, 20):
        js = np.arange(-3, 4)
        ph = np.array([orc.peskin(r - j) for j in js])
        assert abs(ph.sum() - 1) < 1e-15
        assert abs(((r - js) * ph).sum()) < 1e-15
        assert abs((ph ** 2).sum() - 3 / 8) < 1e-15
        even = ph[(js % 2) == 0].sum()
        assert abs(even - 0.5) < 1e-15
    assert orc.peskin(2.0) == 0 and orc.peskin(2.5) == 0 and orc.peskin(-2.0) == 0
    assert abs(orc.peskin(1.0 - 1e-12) - orc.peskin(1.0 + 1e-12)) < 1e-10
    assert orc.peskin(0.3) == orc.peskin(-0.3)


@pytest.mark.parametrize("kind", [0, 1])
def test_stencils_exact_on_quadratics(orc, kind):
    """The isotropic gradient and Laplacian are exact on quadratic fields
    (away from the periodic seam)."""
    n = 12
    p = dict(lattice=kind, nx=n, ny=n, nz=n if kind else 1, kappa=[0.02] * 3, alpha=1.0)
    s = orc.Sim(p)
    D = s.D
    g = np.random.default_rng(5)
    A = g.normal(size=(D, D))
    A = A + A.T
    b = g.normal(size=D)
    grids = np.meshgrid(*([np.arange(n, dtype=float)] * D), indexing="ij")[::-1]  # x, y, (z)
    X = np.stack(grids, axis=-1)  # shape (..., D) with component 0 = x
    q = 0.5 * np.einsum("...a,ab,...b->...", X, A, X) + X @ b
    grad, lap = s.grad_lap(q)
    inner = tuple(slice(1, n - 1) for _ in range(D))
    ref_grad = X @ A + b
    np.testing.assert_allclose(grad[inner], ref_grad[inner], atol=1e-9)
    np.testing.assert_allclose(lap[inner], np.trace(A), atol=1e-9)


def test_stencil_wall_mirror(orc):
    """Walls: the ghost row mirrors the first fluid row, so a field that
    depends on y only has zero normal gradient contribution from the ghost
    (zero-flux condition, eq. NaturalBCs)."""
    p = dict(lattice=0, nx=6, ny=10, wall_y=1, kappa=[0.02] * 3, alpha=1.0)
    s = orc.Sim(p)
    y = np.arange(10, dtype=float)[:, None] * np.ones((1, 6))
    q = y ** 2
    grad, lap = s.grad_lap(q)
    # row 0: neighbours are row 1 and the mirror of row 0
    assert abs(grad[0, 0, 1] - 0.5 * (1.0 - 0.0)) < 1e-12
    assert abs(lap[0, 0] - (1.0 - 0.0)) < 1e-12
    assert abs(grad[9, 0, 1] - 0.5 * (81.0 - 64.0)) < 1e-12


def _C_of(rho, phi, psi):
    """eq. VariableTransform inverted."""
    return np.array([(rho + phi - psi) / 2, (rho - phi - psi) / 2, psi])


def _fb(kap, rho, phi, psi):
    """bulk Landau energy of eq. LandauFE (without the ideal-gas term)."""
    C = _C_of(rho, phi, psi)
    return sum(0.5 * k * c * c * (1 - c) ** 2 for k, c in zip(kap, C))


def test_mu_bulk_is_derivative_of_free_energy(orc):
    """Appendix A: with zero Laplacians the chemical potentials are the
    derivatives of the bulk free energy with respect to rho, phi, psi
    (mu_rho without its ideal-gas part), by central differences."""
    kap = [0.013, 0.029, 0.041]
    p = dict(lattice=0, nx=1, ny=1, kappa=kap, alpha=1.3, kappa_c=0.0)
    g = np.random.default_rng(6)
    h = 1e-5
    for _ in range(20):
        q = np.array([g.uniform(0.8, 1.2), g.uniform(-1, 1), g.uniform(0, 1)])
        mu = orc.mu(p, *q, 0.0, 0.0, 0.0, 0.0)
        for a in range(3):
            e = np.zeros(3)
            e[a] = h
            d = (_fb(kap, *(q + e)) - _fb(kap, *(q - e))) / (2 * h)
            assert abs(mu[a] - d) < 1e-9, (a, mu[a], d)


def test_mu_gradient_part_is_variational(orc):
    """Appendix A: the Laplacian part of mu_q is the variational derivative of
    f_grad = sum alpha^2 kappa_m / 2 |grad C_m|^2, i.e.
    -alpha^2 sum_m kappa_m (dC_m/dq) lap C_m with lap C_m = sum_q' (dC_m/dq') lap q'."""
    kap = np.array([0.013, 0.029, 0.041])
    al = 1.7
    p = dict(lattice=0, nx=1, ny=1, kappa=list(kap), alpha=al, kappa_c=0.0)
    J = np.array([[0.5, 0.5, -0.5], [0.5, -0.5, -0.5], [0.0, 0.0, 1.0]])  # dC_m/dq
    g = np.random.default_rng(7)
    for _ in range(10):
        q = np.array([1.0, g.uniform(-1, 1), g.uniform(0, 1)])
        lap = g.normal(size=3) * 0.01
        mu0 = orc.mu(p, *q, 0.0, 0.0, 0.0, 0.0)
        mu1 = orc.mu(p, *q, *lap, 0.0)
        lapC = J @ lap
        ref = -al ** 2 * (J.T @ (kap * lapC))
        np.testing.assert_allclose(mu1 - mu0, ref, atol=1e-15)


def test_mu_coupling_term(orc):
    """Sec. 3.1: mu_psi' = mu_psi + kappa_c (psi - I) from eq. CouplingE."""
    p = dict(lattice=0, nx=1, ny=1, kappa=[0.01, 0.02, 0.03], alpha=1.0, kappa_c=0.05)
    a = orc.mu(p, 1.0, 0.2, 0.3, 0.01, 0.02, 0.03, 0.0)
    b = orc.mu(p, 1.0, 0.2, 0.3, 0.01, 0.02, 0.03, 0.8)
    assert a[0] == b[0] and a[1] == b[1]
    assert abs((a[2] - b[2]) - 0.05 * 0.8) < 1e-16
