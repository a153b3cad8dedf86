"""Pins of the oracle's membrane mechanics (Sec. 3.2), coupling profile and
coupling force (Sec. 2.5, eqs. Iprofile, DiscreteCE, DiscreteCF) and IBM
transfer operators (Sec. 3.3) against closed forms, finite-difference
gradients of the oracle's own energies, and invariants."""
import numpy as np
import pytest

from paper_1906_03065_amd import workloads as W


def _ring(n, R, noise, seed):
    g = np.random.default_rng(seed)
    X = W.circle_markers(3.0, -2.0, R, n) + g.normal(scale=noise, size=(n, 2))
    return X


def _rest(X):
    return np.linalg.norm(np.roll(X, -1, axis=0) - X, axis=1)


def test_ring_forces_are_energy_gradients(orc):
    """eqs. DiscreteSF, DiscreteBF: F = -dE/dX, checked by central differences
    of the discrete energies of eqs. DiscreteSE and DiscreteBE."""
    X0 = _ring(17, 6.0, 0.0, 0)
    rest = _rest(X0) * np.random.default_rng(1).uniform(0.9, 1.1, 17)
    X = _ring(17, 6.0, 0.4, 2)
    ks, kb = 0.3, 0.07
    F, es, eb = orc.ring_forces(X, rest, ks, kb)
    h = 1e-6
    G = np.zeros_like(X)
    for l in range(len(X)):
        for a in range(2):
            Xp = X.copy(); Xp[l, a] += h
            Xm = X.copy(); Xm[l, a] -= h
            _, e1, b1 = orc.ring_forces(Xp, rest, ks, kb)
            _, e0, b0 = orc.ring_forces(Xm, rest, ks, kb)
            G[l, a] = ((e1 + b1) - (e0 + b0)) / (2 * h)
    np.testing.assert_allclose(F, -G, atol=1e-8 * np.abs(F).max())


def test_ring_forces_free_of_net_force_and_torque(orc):
    """Internal forces of eqs. DiscreteSE/BE depend only on relative
    positions and are rotation invariant: zero sum and zero torque."""
    X = _ring(40, 8.0, 0.3, 3)
    F, _, _ = orc.ring_forces(X, _rest(_ring(40, 7.0, 0.0, 0)), 0.1, 0.01)
    assert np.abs(F.sum(0)).max() < 1e-14
    torque = (X[:, 0] * F[:, 1] - X[:, 1] * F[:, 0]).sum()
    assert abs(torque) < 1e-13


@pytest.mark.parametrize("n", [8, 64, 128])
def test_regular_polygon_energies(orc, n):
    """Regular N-gon of radius R: every turning angle is 2 pi/N, so with
    dtheta = 2 arccos y and ds' = 2 l (eqs. DiscreteBE, DiscreteTheta,
    DiscreteArcLength): E_b = kb pi^2 / (N R sin(pi/N)).  Stretched to R':
    E_s = ks/2 N (l'/ds - 1)^2 ds with l = 2 R sin(pi/N)."""
    R, ks, kb = 20.0, 0.01, 1e-4
    X = W.circle_markers(0.0, 0.0, R, n)
    rest = _rest(X)
    F, es, eb = orc.ring_forces(X, rest, ks, kb)
    assert abs(es) < 1e-30
    np.testing.assert_allclose(eb, kb * np.pi ** 2 / (n * R * np.sin(np.pi / n)), rtol=1e-12)
    X2 = W.circle_markers(0.0, 0.0, 1.1 * R, n)
    _, es2, _ = orc.ring_forces(X2, rest, ks, kb)
    ds = 2 * R * np.sin(np.pi / n)
    np.testing.assert_allclose(es2, ks / 2 * n * (1.1 * ds / ds - 1) ** 2 * ds, rtol=1e-12)
    # forces on a regular polygon are radial
    rad = X / np.linalg.norm(X, axis=1, keepdims=True)
    tang = np.stack([-rad[:, 1], rad[:, 0]], 1)
    assert np.abs((F * tang).sum(1)).max() < 1e-15


def test_mesh_forces_are_energy_gradients(orc):
    """3D edge-spring + dihedral membrane law: F = -dE/dX by central
    differences, zero net force and torque."""
    V, T = W.icosphere(1)
    g = np.random.default_rng(4)
    X0 = V * 3.0
    edges = set()
    for t in T:
        for k in range(3):
            a, b = t[k], t[(k + 1) % 3]
            edges.add((min(a, b), max(a, b)))
    # the oracle orders edges by first appearance over triangles
    order = []
    seen = set()
    for t in T:
        for k in range(3):
            a, b = int(t[k]), int(t[(k + 1) % 3])
            key = (min(a, b), max(a, b))
            if key not in seen:
                seen.add(key)
                order.append(key)
    rest = np.array([np.linalg.norm(X0[b] - X0[a]) for a, b in order])
    X = X0 + g.normal(scale=0.2, size=X0.shape)
    ks, kb = 0.2, 0.05
    F, es, eb = orc.mesh_forces(X, T, rest, ks, kb)
    h = 1e-6
    G = np.zeros_like(X)
    for v in range(len(X)):
        for a in range(3):
            Xp = X.copy(); Xp[v, a] += h
            Xm = X.copy(); Xm[v, a] -= h
            _, e1, b1 = orc.mesh_forces(Xp, T, rest, ks, kb)
            _, e0, b0 = orc.mesh_forces(Xm, T, rest, ks, kb)
            G[v, a] = ((e1 + b1) - (e0 + b0)) / (2 * h)
    np.testing.assert_allclose(F, -G, atol=1e-8 * np.abs(F).max())
    assert np.abs(F.sum(0)).max() < 1e-13
    assert np.abs(np.cross(X, F).sum(0)).max() < 1e-12
    # unstretched, flat-angle-free sphere: no strain energy
    _, es0, eb0 = orc.mesh_forces(X0, T, rest, ks, kb)
    assert es0 < 1e-28 and eb0 > 0


def _sim_with_ring(orc, n=40, R=9.0, centre=(20.3, 19.7), nx=40, ny=40, alpha=1.0, kc=0.01,
                   wall_y=0, rc=0.0):
    p = W.base_params(nx, ny, wall_y=wall_y, kappa=(0.02, 0.02, 0.02), alpha=alpha, kappa_c=kc,
                      r_cut=rc)
    s = orc.Sim(p)
    X = W.circle_markers(centre[0], centre[1], R, n)
    s.add_membrane(X, None, 0.0, 0.0)
    return s, X, p


def test_coupling_profile_matches_circle(orc):
    """eq. Iprofile on a fine polygon approximates the tanh profile of the
    exact circle distance (the polygon sits inside the circle by at most
    R (1 - cos(pi/N))); deep inside I = 1, far outside I = 0."""
    n, R, al = 256, 9.0, 1.0
    s, X, _ = _sim_with_ring(orc, n=n, R=R, alpha=al)
    psi = np.zeros(s.shape)
    I, Fc, Ec = s.coupling(psi)
    y, x = np.meshgrid(np.arange(40.0), np.arange(40.0), indexing="ij")
    d = R - np.hypot(x - 20.3, y - 19.7)
    ref = W.tanh_profile(d, al)
    sag = R * (1 - np.cos(np.pi / n))
    assert np.abs(I - ref).max() < 0.26 * sag / al + 1e-12
    assert I[20, 20] == 1.0 - 0.0 or abs(I[20, 20] - W.tanh_profile(R - 0.7, al)) < 1e-2
    assert I[0, 0] < 1e-5
    # the energy reported is kappa_c/2 sum (psi - I)^2
    np.testing.assert_allclose(Ec, 0.5 * 0.01 * (I ** 2).sum(), rtol=1e-13)


def test_coupling_profile_without_band(orc):
    """r_cut <= 0: no band, eq. Iprofile everywhere.  Between 18 and 30
    lattice units outside a fine ring the profile is the tanh tail of the
    circle distance (relative error of the order of the polygon's sag over
    alpha); with a band of 17 the same nodes are exactly 0, and inside the
    band both agree exactly."""
    n, R, c, N = 256, 6.0, (40.3, 39.6), 80
    p0 = W.base_params(N, N, kappa=(0.02,) * 3, alpha=1.0, kappa_c=0.01, r_cut=0.0)
    p17 = dict(p0, r_cut=17.0)
    X = W.circle_markers(c[0], c[1], R, n)
    out = []
    for p in (p0, p17):
        s = orc.Sim(p)
        s.add_membrane(X, None, 0.0, 0.0)
        out.append(s.coupling(np.zeros((N, N)))[0])
    I0, I17 = out
    y, x = np.meshgrid(np.arange(float(N)), np.arange(float(N)), indexing="ij")
    d = R - np.hypot(x - c[0], y - c[1])
    tail = (d < -18.0) & (d > -30.0)
    ref = W.tanh_profile(d, 1.0)
    assert tail.sum() > 1000
    assert np.all(I0[tail] > 0.0) and np.all(I17[tail] == 0.0)
    assert np.abs(I0[tail] / ref[tail] - 1.0).max() < 3.0 * R * (1 - np.cos(np.pi / n))
    band = d > -16.5
    assert np.array_equal(I0[band], I17[band])


def test_coupling_profiles_add(orc):
    """Several membranes: their profiles add (each capsule encloses fluid 3)."""
    p = W.base_params(60, 30, kappa=(0.02,) * 3, alpha=1.0, kappa_c=0.01)
    s = orc.Sim(p)
    A = W.circle_markers(15.2, 14.6, 6.0, 40)
    B = W.circle_markers(44.7, 15.1, 7.0, 48)
    s.add_membrane(A, None, 0, 0)
    s.add_membrane(B, None, 0, 0)
    sa = orc.Sim(p); sa.add_membrane(A, None, 0, 0)
    sb = orc.Sim(p); sb.add_membrane(B, None, 0, 0)
    z = np.zeros(s.shape)
    I, _, _ = s.coupling(z)
    Ia, _, _ = sa.coupling(z)
    Ib, _, _ = sb.coupling(z)
    np.testing.assert_allclose(I, Ia + Ib, atol=1e-15)


def test_coupling_force_is_energy_gradient(orc):
    """eq. DiscreteCF with A7's reading of the sign: the coupling force is
    -dE_c/dX_l of eq. DiscreteCE at fixed psi, by central differences."""
    n, R = 24, 6.0
    p = W.base_params(24, 24, kappa=(0.02,) * 3, alpha=1.0, kappa_c=0.05)
    g = np.random.default_rng(8)
    X = W.circle_markers(11.6, 12.3, R, n) + g.normal(scale=0.15, size=(n, 2))
    y, x = np.meshgrid(np.arange(24.0), np.arange(24.0), indexing="ij")
    psi = W.tanh_profile(R + 0.8 - np.hypot(x - 12.0, y - 12.0), 1.0)

    def energy(Xm):
        s = orc.Sim(p)
        s.add_membrane(Xm, None, 0, 0)
        return s.coupling(psi)

    _, Fc, _ = energy(X)
    h = 1e-6
    G = np.zeros_like(X)
    for l in range(n):
        for a in range(2):
            Xp = X.copy(); Xp[l, a] += h
            Xm = X.copy(); Xm[l, a] -= h
            G[l, a] = (energy(Xp)[2] - energy(Xm)[2]) / (2 * h)
    np.testing.assert_allclose(Fc, -G, atol=2e-6 * np.abs(Fc).max())


def test_spread_interp_adjoint_and_moments(orc):
    """eqs. Spreading and Interpolation use the same kernel, so they are
    adjoint: sum_x f_IB . v = sum_l F_l . U_l.  The spread total equals the
    sum of marker forces and a linear field is interpolated exactly."""
    p = W.base_params(32, 24, kappa=(0.02,) * 3, alpha=1.0)
    s = orc.Sim(p)
    g = np.random.default_rng(9)
    X = g.uniform([3, 3], [28, 20], size=(30, 2))
    F = g.normal(size=(30, 2))
    v = g.normal(size=s.shape + (2,))
    fib = s.spread(X, F)
    U = s.interp(X, v)
    assert abs((fib * v).sum() - (F * U).sum()) < 1e-12
    np.testing.assert_allclose(fib.reshape(-1, 2).sum(0), F.sum(0), atol=1e-13)
    y, x = np.meshgrid(np.arange(24.0), np.arange(32.0), indexing="ij")
    lin = np.stack([0.3 * x - 0.2 * y + 1.0, 0.1 * x + 0.5 * y], -1)
    U = s.interp(X, lin)
    ref = np.stack([0.3 * X[:, 0] - 0.2 * X[:, 1] + 1.0, 0.1 * X[:, 0] + 0.5 * X[:, 1]], 1)
    np.testing.assert_allclose(U, ref, atol=1e-12)
    # first moment: sum_x x f_IB = sum_l X_l F_l (away from the periodic seam)
    mx = (fib[..., 0] * x).sum()
    assert abs(mx - (F[:, 0] * X[:, 0]).sum()) < 1e-11


def test_spread_skips_nodes_beyond_walls(orc):
    """Walls: stencil nodes outside the fluid are dropped (READING)."""
    p = W.base_params(16, 8, wall_y=1, kappa=(0.02,) * 3, alpha=1.0)
    s = orc.Sim(p)
    X = np.array([[5.3, 0.4]])
    F = np.array([[1.0, 2.0]])
    fib = s.spread(X, F)
    wy = sum(orc.peskin(j - 0.4) for j in range(0, 3))
    np.testing.assert_allclose(fib.reshape(-1, 2).sum(0), F[0] * wy, atol=1e-14)
